"""ctypes binding of include/pdschur.h (argument marshalling only)."""
import atexit
import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBNAME = "libpdschur.so"

PD_OK, PD_ERR_INVALID, PD_ERR_HIP, PD_ERR_OOM, PD_ERR_NOT_SPD, PD_ERR_IR_STALLED, PD_ERR_STATE = \
    0, -1, -2, -3, -4, -5, -6
PD_FP64, PD_FP32_IR, PD_BF16_IR = 0, 1, 2
_NAMES = {0: "PD_OK", -1: "PD_ERR_INVALID", -2: "PD_ERR_HIP", -3: "PD_ERR_OOM",
          -4: "PD_ERR_NOT_SPD", -5: "PD_ERR_IR_STALLED", -6: "PD_ERR_STATE"}


class PDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class pd_mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_tets", C.c_int64), ("rest", C.c_void_p),
                ("tets", C.c_void_p), ("region", C.c_void_p), ("dirichlet", C.c_void_p),
                ("mu", C.c_double), ("density", C.c_double), ("dt", C.c_double),
                ("mu_prime", C.c_double), ("sigma_min", C.c_double), ("sigma_max", C.c_double),
                ("interior_order", C.c_int32), ("nd_leaf", C.c_int32)]


class pd_solve_info(C.Structure):
    _fields_ = [("ir_iters", C.c_int32), ("bad_pivot", C.c_int32), ("fell_back", C.c_int32),
                ("reserved", C.c_int32), ("rel_residual", C.c_double)]


_P = C.c_void_p
_SIGS = {
    "pd_schur_build": [C.POINTER(pd_mesh), _P, C.POINTER(_P)],
    "pd_query": [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                 C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
    "pd_region_nodes": [_P, _P],
    "pd_get_schur": [_P, _P],
    "pd_region_gather": [_P, _P, _P],
    "pd_local_step_full": [_P, _P, _P, _P, C.c_int],
    "pd_set_inertia_target": [_P, _P],
    "pd_time_step_advance": [_P, _P, _P, _P, _P],
    "pd_condense_rhs": [_P, _P, _P],
    "pd_detect_spheres": [_P, C.c_int32, _P, C.c_int32, _P, C.c_double, _P, _P, _P, _P, _P],
    "pd_collision_update": [_P, C.c_int32, _P, _P, _P, _P, _P, _P],
    "pd_detect_pairs": [_P, C.c_int32, _P, C.c_double, _P, _P, _P, _P, _P],
    "pd_embed_points": [_P, C.c_int32, _P, C.c_int32, _P, _P, _P, _P, _P],
    "pd_detect_embedded_spheres": [_P, C.c_int32, _P, _P, C.c_int32, _P, C.c_double, _P, _P, _P,
                                   _P, _P],
    "pd_detect_levelset": [_P, C.c_int32, _P, _P, _P, C.c_int32, _P, _P, _P, _P, C.c_double, _P,
                           _P, _P, _P, _P],
    "pd_local_step_region": [_P, _P, _P, _P, C.c_int],
    "pd_assemble_rhs": [_P, _P, _P, _P, _P],
    "pd_global_solve": [_P, _P, _P, C.c_int, C.POINTER(pd_solve_info)],
    "pd_inner_update": [_P, _P, _P, _P, _P],
    "pd_backsub": [_P, _P, _P],
    "pd_mlp_create": [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, _P,
                      C.POINTER(_P)],
    "pd_mlp_get_params": [_P, _P],
    "pd_mlp_forward": [_P, _P, _P, C.c_int32],
    "pd_mlp_train_step": [_P, _P, _P, C.c_int32, C.c_float, C.POINTER(C.c_double), _P],
    "pd_mlp_destroy": [_P],
    "pd_mlp_gather_rows": [_P, _P, C.c_int32, C.c_int32, _P, C.c_int32, C.c_int32, C.c_float, _P],
    "pd_mlp_abs_mean": [_P, _P, C.c_int64, C.POINTER(C.c_double)],
    "pd_chol_create": [C.c_int64, _P, C.POINTER(_P)],
    "pd_chol_factor": [_P, _P, C.c_int64, C.c_int64, C.c_int32, C.POINTER(C.c_int32)],
    "pd_chol_destroy": [_P],
    "pd_nd_analyse": [C.POINTER(pd_mesh), C.c_int32, _P, _P, _P, _P, _P, _P],
    "pd_dataflow_task": [C.c_int64, C.c_int32, C.c_int64, C.POINTER(C.c_int32),
                         C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int64)],
    "pd_chol_factor_noalloc": [_P, C.c_int64, C.c_int64, C.c_int32, _P, C.POINTER(C.c_int32)],
    "pd_displacement_change": [_P, _P, _P, _P],
    "pd_warmstart_input": [_P, _P, _P, C.c_float, C.c_int32, _P, _P, _P],
    "pd_region_add_f32": [_P, _P, C.c_double, _P],
    "pd_warmstart_apply": [_P, _P, C.c_double, _P, _P, _P],
    "pd_warmstart_target": [_P, _P, _P, _P, C.c_float, _P],
    "pd_set_stream": [_P, _P],
    "pd_use_stream": [_P, _P],
    "pd_factor": [_P, C.c_int32, C.c_int32],
    "pd_set_refinement": [_P, C.c_int32, C.c_double, C.c_int32],
    "pd_set_timing": [_P, C.c_int],
    "pd_get_timings": [_P, _P, _P],
    "pd_destroy": [_P],
}
PHASES = ["local_full", "condense", "detect", "collision", "local_region", "assemble",
          "hbuild", "factor", "solve", "inner_update", "backsub"]

_lib = None

# Handles (contexts, factorizations, networks) still open.  They are closed by
# an exit handler registered after torch, so it runs before torch's own exit
# handlers and before the HIP runtime and any profiler tool are torn down;
# after it, __del__ never calls into the library (objects collected during
# interpreter teardown would otherwise free device memory and events after the
# runtime is gone).
_open_handles = weakref.WeakSet()
_exiting = False


def _close_all_at_exit():
    global _exiting
    for h in list(_open_handles):
        try:
            h.close()
        except Exception:
            pass
    _exiting = True


class _Handle:
    """Base of the objects owning a library handle: explicit close(), also as
    a context manager; __del__ closes only before interpreter exit."""

    def _register(self):
        _open_handles.add(self)

    def close(self):
        raise NotImplementedError

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass


def library_path():
    return os.path.join(_HERE, _LIBNAME)


def load_library():
    """Load libpdschur.so; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not built; run paper_2008_01541_amd/build.py "
                           "(or __graft_entry__.build())")
    lib = C.CDLL(path)
    for name, args in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.pd_last_error.argtypes = [_P]
    lib.pd_last_error.restype = C.c_char_p
    import torch  # noqa: F401  (its exit handlers must run after ours)
    atexit.register(_close_all_at_exit)
    _lib = lib
    return lib


def _ptr(t, dtype=None, numel=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (or None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return t.data_ptr()


def nd_analyse(rest, tets, region, dirichlet, leaf=256):
    """pd_nd_analyse: nested-dissection ordering and boundary sets of the
    interior nodes (host only).  Returns a dict with n1, elim [n1], first
    [ns+1], parent [ns], bptr [ns+1] and bkey [nb] (numpy arrays)."""
    lib = load_library()
    rest = np.ascontiguousarray(rest, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    region = np.ascontiguousarray(region, dtype=np.uint8)
    dirichlet = np.ascontiguousarray(dirichlet, dtype=np.uint8)
    mesh = pd_mesh(rest.shape[1], tets.shape[1], rest.ctypes.data, tets.ctypes.data,
                   region.ctypes.data, dirichlet.ctypes.data, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1,
                   int(leaf))
    sizes = np.zeros(3, dtype=np.int64)
    st = lib.pd_nd_analyse(C.byref(mesh), int(leaf), sizes.ctypes.data, None, None, None, None,
                           None)
    if st != PD_OK:
        raise PDError(st, "pd_nd_analyse failed")
    n1, ns, nb = (int(v) for v in sizes)
    out = dict(n1=n1, elim=np.zeros(n1, np.int32), first=np.zeros(ns + 1, np.int32),
               parent=np.zeros(ns, np.int32), bptr=np.zeros(ns + 1, np.int64),
               bkey=np.zeros(max(nb, 1), np.int32))
    st = lib.pd_nd_analyse(C.byref(mesh), int(leaf), sizes.ctypes.data, out["elim"].ctypes.data,
                           out["first"].ctypes.data, out["parent"].ctypes.data,
                           out["bptr"].ctypes.data, out["bkey"].ctypes.data)
    if st != PD_OK:
        raise PDError(st, "pd_nd_analyse failed")
    out["bkey"] = out["bkey"][:nb]
    return out


class PDContext(_Handle):
    """One built mesh (pd_schur_build) and its per-iteration entry points."""

    def __init__(self, rest, tets, region, dirichlet, mu, stream=None, density=0.0, dt=0.0,
                 mu_prime=0.0, sigma_min=0.0, sigma_max=0.0, interior="levels", nd_leaf=0):
        import torch
        lib = load_library()
        self._lib = lib
        rest = np.ascontiguousarray(rest, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        region = np.ascontiguousarray(region, dtype=np.uint8)
        dirichlet = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        n = rest.shape[1]
        T = tets.shape[1]
        if rest.shape != (3, n) or tets.shape != (4, T) or region.shape != (n,) or \
                dirichlet.shape != (n,):
            raise ValueError("mesh arrays have inconsistent shapes")
        self._keep = (rest, tets, region, dirichlet)
        if interior not in ("levels", "nd"):
            raise ValueError("interior must be 'levels' or 'nd'")
        mesh = pd_mesh(n, T, rest.ctypes.data, tets.ctypes.data, region.ctypes.data,
                       dirichlet.ctypes.data, float(mu), float(density), float(dt),
                       float(mu_prime), float(sigma_min), float(sigma_max),
                       1 if interior == "nd" else 0, int(nd_leaf))
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        ctx = C.c_void_p()
        st = lib.pd_schur_build(C.byref(mesh), C.c_void_p(stream.cuda_stream), C.byref(ctx))
        if st != PD_OK:
            raise PDError(st, lib.pd_last_error(None).decode())
        self._ctx = ctx
        self._register()
        m, n1, nb, na, nl = (C.c_int64() for _ in range(5))
        self._chk(lib.pd_query(ctx, C.byref(m), C.byref(n1), C.byref(nb), C.byref(na),
                               C.byref(nl)))
        self.n, self.m, self.n1 = n, m.value, n1.value
        self.n_beta, self.n_alpha, self.n_levels = nb.value, na.value, nl.value
        ids = np.empty(self.m, dtype=np.int32)
        self._chk(lib.pd_region_nodes(ctx, ids.ctypes.data))
        self.region_ids = ids

    def _chk(self, st):
        if st != PD_OK:
            raise PDError(st, self._lib.pd_last_error(self._ctx).decode())

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.pd_destroy(self._ctx)
            self._ctx = None

    # --- entry points (names as in the C ABI) ------------------------------
    def get_schur(self, S):
        import torch
        self._chk(self._lib.pd_get_schur(self._ctx, _ptr(S, torch.float64, self.m * self.m, "S")))

    def region_gather(self, x, x2):
        import torch
        self._chk(self._lib.pd_region_gather(self._ctx, _ptr(x, torch.float64, 3 * self.n, "x"),
                                             _ptr(x2, torch.float64, 3 * self.m, "x2")))

    def local_step_full(self, x, f, R_alpha=None, rot_fp32=False):
        import torch
        rdt = torch.float32 if rot_fp32 else torch.float64
        self._chk(self._lib.pd_local_step_full(
            self._ctx, _ptr(x, torch.float64, 3 * self.n, "x"),
            _ptr(R_alpha, rdt, 9 * self.n_alpha, "R_alpha"),
            _ptr(f, torch.float64, 3 * self.n, "f"), 1 if rot_fp32 else 0))

    def set_inertia_target(self, y):
        import torch
        self._chk(self._lib.pd_set_inertia_target(
            self._ctx, None if y is None else _ptr(y, torch.float64, 3 * self.n, "y")))

    def time_step_advance(self, x, x_prev, v, y):
        import torch
        self._chk(self._lib.pd_time_step_advance(
            self._ctx, _ptr(x, torch.float64, 3 * self.n, "x"),
            _ptr(x_prev, torch.float64, 3 * self.n, "x_prev"),
            _ptr(v, torch.float64, 3 * self.n, "v"), _ptr(y, torch.float64, 3 * self.n, "y")))

    def condense_rhs(self, f, y2):
        import torch
        self._chk(self._lib.pd_condense_rhs(self._ctx, _ptr(f, torch.float64, 3 * self.n, "f"),
                                            _ptr(y2, torch.float64, 3 * self.m, "y2")))

    def detect_spheres(self, prox, spheres, k, x2, idx, w, c, t):
        import torch
        npx = prox.numel()
        nsph = spheres.numel() // 4
        self._chk(self._lib.pd_detect_spheres(
            self._ctx, npx, _ptr(prox, torch.int32, npx, "prox"), nsph,
            _ptr(spheres, torch.float64, 4 * nsph, "spheres"), float(k),
            _ptr(x2, torch.float64, 3 * self.m, "x2"), _ptr(idx, torch.int32, 8 * npx, "idx"),
            _ptr(w, torch.float64, 8 * npx, "w"), _ptr(c, torch.float64, npx, "c"),
            _ptr(t, torch.float64, 3 * npx, "t")))

    def detect_pairs(self, pairs, k, x2, idx, w, c, t):
        import torch
        npr = pairs.numel() // 2
        self._chk(self._lib.pd_detect_pairs(
            self._ctx, npr, _ptr(pairs, torch.int32, 2 * npr, "pairs"), float(k),
            _ptr(x2, torch.float64, 3 * self.m, "x2"), _ptr(idx, torch.int32, 8 * npr, "idx"),
            _ptr(w, torch.float64, 8 * npr, "w"), _ptr(c, torch.float64, npr, "c"),
            _ptr(t, torch.float64, 3 * npr, "t")))

    def embed_points(self, pts, cand, pos, tet, eidx, ew):
        """pd_embed_points: pts [3][n], cand [4][nc] region-local, pos [3][m]."""
        import torch
        n = pts.numel() // 3
        nc = cand.numel() // 4
        self._chk(self._lib.pd_embed_points(
            self._ctx, n, _ptr(pts, torch.float64, 3 * n, "pts"), nc,
            _ptr(cand, torch.int32, 4 * nc, "cand"), _ptr(pos, torch.float64, 3 * self.m, "pos"),
            _ptr(tet, torch.int32, n, "tet"), _ptr(eidx, torch.int32, 4 * n, "eidx"),
            _ptr(ew, torch.float64, 4 * n, "ew")))

    def detect_embedded_spheres(self, eidx, ew, spheres, k, x2, idx, w, c, t):
        import torch
        npx = eidx.numel() // 4
        nsph = spheres.numel() // 4
        self._chk(self._lib.pd_detect_embedded_spheres(
            self._ctx, npx, _ptr(eidx, torch.int32, 4 * npx, "eidx"),
            _ptr(ew, torch.float64, 4 * npx, "ew"), nsph,
            _ptr(spheres, torch.float64, 4 * nsph, "spheres"), float(k),
            _ptr(x2, torch.float64, 3 * self.m, "x2"), _ptr(idx, torch.int32, 8 * npx, "idx"),
            _ptr(w, torch.float64, 8 * npx, "w"), _ptr(c, torch.float64, npx, "c"),
            _ptr(t, torch.float64, 3 * npx, "t")))

    def detect_levelset(self, eidx, ew, prox_body, cand, cand_phi, cand_body, rest2, k, x2,
                        idx, w, c, t):
        import torch
        npx = eidx.numel() // 4
        nc = cand.numel() // 4
        self._chk(self._lib.pd_detect_levelset(
            self._ctx, npx, _ptr(eidx, torch.int32, 4 * npx, "eidx"),
            _ptr(ew, torch.float64, 4 * npx, "ew"), _ptr(prox_body, torch.int32, npx, "prox_body"),
            nc, _ptr(cand, torch.int32, 4 * nc, "cand"),
            _ptr(cand_phi, torch.float64, 4 * nc, "cand_phi"),
            _ptr(cand_body, torch.int32, nc, "cand_body"),
            _ptr(rest2, torch.float64, 3 * self.m, "rest2"), float(k),
            _ptr(x2, torch.float64, 3 * self.m, "x2"), _ptr(idx, torch.int32, 8 * npx, "idx"),
            _ptr(w, torch.float64, 8 * npx, "w"), _ptr(c, torch.float64, npx, "c"),
            _ptr(t, torch.float64, 3 * npx, "t")))

    def collision_update(self, idx, w, c, t, x2, f_col):
        import torch
        npen = c.numel()
        self._chk(self._lib.pd_collision_update(
            self._ctx, npen, _ptr(idx, torch.int32, 8 * npen, "idx"),
            _ptr(w, torch.float64, 8 * npen, "w"), _ptr(c, torch.float64, npen, "c"),
            _ptr(t, torch.float64, 3 * npen, "t"), _ptr(x2, torch.float64, 3 * self.m, "x2"),
            _ptr(f_col, torch.float64, 3 * self.m, "f_col")))

    def local_step_region(self, x2, f_beta, R_beta=None, rot_fp32=False):
        import torch
        rdt = torch.float32 if rot_fp32 else torch.float64
        self._chk(self._lib.pd_local_step_region(
            self._ctx, _ptr(x2, torch.float64, 3 * self.m, "x2"),
            _ptr(R_beta, rdt, 9 * self.n_beta, "R_beta"),
            _ptr(f_beta, torch.float64, 3 * self.m, "f_beta"), 1 if rot_fp32 else 0))

    def assemble_rhs(self, ft, f_beta, f_col, g):
        import torch
        self._chk(self._lib.pd_assemble_rhs(
            self._ctx, _ptr(ft, torch.float64, 3 * self.m, "ft"),
            _ptr(f_beta, torch.float64, 3 * self.m, "f_beta"),
            _ptr(f_col, torch.float64, 3 * self.m, "f_col"), _ptr(g, torch.float64, 3 * self.m, "g")))

    def global_solve(self, g, u, prec=PD_FP64, want_info=False):
        import torch
        info = pd_solve_info() if want_info else None
        st = self._lib.pd_global_solve(self._ctx, _ptr(g, torch.float64, 3 * self.m, "g"),
                                       _ptr(u, torch.float64, 3 * self.m, "u"), int(prec),
                                       C.byref(info) if info is not None else None)
        if info is not None:
            res = dict(ir_iters=info.ir_iters, bad_pivot=info.bad_pivot,
                       fell_back=info.fell_back, rel_residual=info.rel_residual, status=st)
            if st != PD_OK and st != PD_ERR_IR_STALLED:
                self._chk(st)
            return res
        self._chk(st)
        return None

    def set_refinement(self, max_steps=100, tol=1e-8, fallback=True):
        """Settings of the refined solves (pd_set_refinement)."""
        self._chk(self._lib.pd_set_refinement(self._ctx, int(max_steps), float(tol),
                                              int(fallback)))

    def factor(self, n_workgroups=0, overlap_forward=False):
        """FP64 factorization of H ahead of global_solve (pd_factor); with
        overlap_forward the next global_solve may be enqueued on another stream
        while it runs."""
        self._chk(self._lib.pd_factor(self._ctx, int(n_workgroups), 1 if overlap_forward else 0))

    def inner_update(self, u2, x2, delta2, ft):
        import torch
        self._chk(self._lib.pd_inner_update(
            self._ctx, _ptr(u2, torch.float64, 3 * self.m, "u2"),
            _ptr(x2, torch.float64, 3 * self.m, "x2"),
            _ptr(delta2, torch.float64, 3 * self.m, "delta2"),
            _ptr(ft, torch.float64, 3 * self.m, "ft")))

    def displacement_change(self, x, x_prev):
        """(||x - x_prev||, ||x - X||) over the free nodes (synchronizes)."""
        import torch
        out = np.zeros(2, dtype=np.float64)
        self._chk(self._lib.pd_displacement_change(
            self._ctx, _ptr(x, torch.float64, 3 * self.n, "x"),
            _ptr(x_prev, torch.float64, 3 * self.n, "x_prev"), out.ctypes.data))
        return float(out[0]), float(out[1])

    def warmstart_input(self, x2, x2_prev, scale, prox, cpen, out):
        import torch
        npx = prox.numel()
        self._chk(self._lib.pd_warmstart_input(
            self._ctx, _ptr(x2, torch.float64, 3 * self.m, "x2"),
            _ptr(x2_prev, torch.float64, 3 * self.m, "x2_prev"), float(scale), npx,
            _ptr(prox, torch.int32, npx, "prox"), _ptr(cpen, torch.float64, npx, "c"),
            _ptr(out, torch.float32, 4 * self.m, "out")))

    def warmstart_apply(self, d2, scale, x, x2_prev1=None, x2_prev2=None):
        import torch
        self._chk(self._lib.pd_warmstart_apply(
            self._ctx, _ptr(d2, torch.float32, 3 * self.m, "d2"), float(scale),
            _ptr(x2_prev1, torch.float64, 3 * self.m, "x2_prev1"),
            _ptr(x2_prev2, torch.float64, 3 * self.m, "x2_prev2"),
            _ptr(x, torch.float64, 3 * self.n, "x")))

    def warmstart_target(self, x2, x2_prev1, x2_prev2, scale, out):
        import torch
        self._chk(self._lib.pd_warmstart_target(
            self._ctx, _ptr(x2, torch.float64, 3 * self.m, "x2"),
            _ptr(x2_prev1, torch.float64, 3 * self.m, "x2_prev1"),
            _ptr(x2_prev2, torch.float64, 3 * self.m, "x2_prev2"), float(scale),
            _ptr(out, torch.float32, 3 * self.m, "out")))

    def region_add_f32(self, d2, scale, x):
        import torch
        self._chk(self._lib.pd_region_add_f32(self._ctx, _ptr(d2, torch.float32, 3 * self.m, "d2"),
                                              float(scale), _ptr(x, torch.float64, 3 * self.n, "x")))

    def set_stream(self, stream):
        self._chk(self._lib.pd_set_stream(self._ctx, C.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def use_stream(self, stream):
        """Enqueue later calls on stream without synchronizing (pd_use_stream)."""
        self._chk(self._lib.pd_use_stream(self._ctx, C.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def set_timing(self, on=True):
        self._chk(self._lib.pd_set_timing(self._ctx, 1 if on else 0))

    def get_timings(self):
        """{phase: (total ms, calls)} since the previous call (synchronizes)."""
        ms = np.zeros(len(PHASES), dtype=np.float64)
        cnt = np.zeros(len(PHASES), dtype=np.int64)
        self._chk(self._lib.pd_get_timings(self._ctx, ms.ctypes.data, cnt.ctypes.data))
        return {p: (float(ms[i]), int(cnt[i])) for i, p in enumerate(PHASES)}

    def backsub(self, delta2, x):
        import torch
        self._chk(self._lib.pd_backsub(self._ctx, _ptr(delta2, torch.float64, 3 * self.m, "delta2"),
                                       _ptr(x, torch.float64, 3 * self.n, "x")))


class DenseCholesky(_Handle):
    """Standalone dense FP64 Cholesky (pd_chol_* entry points): in-place
    factorization of a device matrix of order up to n_max."""

    def __init__(self, n_max, stream=None):
        import torch
        lib = load_library()
        self._lib = lib
        if stream is None:
            stream = torch.cuda.current_stream()
        h = C.c_void_p()
        st = lib.pd_chol_create(int(n_max), C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != PD_OK:
            raise PDError(st, "pd_chol_create failed")
        self._h = h
        self._register()
        self.n_max = int(n_max)

    def factor(self, A, n, lda, n_workgroups=0, want_info=True):
        """A: device float64 tensor holding an n x n matrix column-major with
        leading dimension lda (lda * n elements).  Returns the pivot info (0 if
        positive definite) when want_info, else None (enqueue only)."""
        import torch
        ptr = _ptr(A, torch.float64, int(lda) * int(n), "A")
        if not want_info:
            st = self._lib.pd_chol_factor(self._h, ptr, int(lda), int(n), int(n_workgroups), None)
            if st != PD_OK:
                raise PDError(st, "pd_chol_factor failed")
            return None
        info = C.c_int32(0)
        st = self._lib.pd_chol_factor(self._h, ptr, int(lda), int(n), int(n_workgroups),
                                      C.byref(info))
        if st not in (PD_OK, PD_ERR_NOT_SPD):
            raise PDError(st, "pd_chol_factor failed")
        return int(info.value)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pd_chol_destroy(self._h)
            self._h = None


def chol_factor_noalloc(A, n, lda, n_workgroups=0, want_info=True, stream=None):
    """pd_chol_factor_noalloc: the factorization of DenseCholesky.factor with
    the library's static workspace (n <= PD_CHOL_NOALLOC_MAX_N), on `stream`
    (default: torch's current stream).  Returns the pivot info when want_info."""
    import torch
    lib = load_library()
    if stream is None:
        stream = torch.cuda.current_stream()
    ptr = _ptr(A, torch.float64, int(lda) * int(n), "A")
    info = C.c_int32(0)
    st = lib.pd_chol_factor_noalloc(ptr, int(lda), int(n), int(n_workgroups),
                                    C.c_void_p(stream.cuda_stream),
                                    C.byref(info) if want_info else None)
    if st not in (PD_OK, PD_ERR_NOT_SPD) or (st == PD_ERR_NOT_SPD and not want_info):
        raise PDError(st, "pd_chol_factor_noalloc failed")
    return int(info.value) if want_info else None


PD_CHOL_NOALLOC_MAX_N = 8192


class MLP(_Handle):
    """Warm-start network (pd_mlp_* entry points)."""

    def __init__(self, n_in, n_h1, n_h2, n_out, max_batch, params_flat, stream=None):
        import torch
        lib = load_library()
        self._lib = lib
        p = np.ascontiguousarray(params_flat, dtype=np.float32)
        self.shape = (n_in, n_h1, n_h2, n_out)
        self.n_params = n_h1 * n_in + n_h1 + n_h2 * n_h1 + n_h2 + n_out * n_h2 + n_out
        if p.size != self.n_params:
            raise ValueError("parameter vector has the wrong length")
        if stream is None:
            stream = torch.cuda.current_stream()
        h = C.c_void_p()
        st = lib.pd_mlp_create(n_in, n_h1, n_h2, n_out, max_batch, p.ctypes.data,
                               C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != PD_OK:
            raise PDError(st, "pd_mlp_create failed")
        self._h = h
        self._register()
        self.max_batch = max_batch

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pd_mlp_destroy(self._h)
            self._h = None

    def params(self):
        out = np.empty(self.n_params, dtype=np.float32)
        st = self._lib.pd_mlp_get_params(self._h, out.ctypes.data)
        if st != PD_OK:
            raise PDError(st, "pd_mlp_get_params failed")
        return out

    def forward(self, x, y):
        import torch
        B = x.numel() // self.shape[0]
        st = self._lib.pd_mlp_forward(self._h, _ptr(x, torch.float32, B * self.shape[0], "x"),
                                      _ptr(y, torch.float32, B * self.shape[3], "y"), B)
        if st != PD_OK:
            raise PDError(st, "pd_mlp_forward failed")

    def train_step(self, x, target, lr, want_loss=True):
        import torch
        B = x.numel() // self.shape[0]
        loss = C.c_double()
        st = self._lib.pd_mlp_train_step(self._h, _ptr(x, torch.float32, B * self.shape[0], "x"),
                                         _ptr(target, torch.float32, B * self.shape[3], "target"),
                                         B, float(lr), C.byref(loss) if want_loss else None, None)
        if st != PD_OK:
            raise PDError(st, "pd_mlp_train_step failed")
        return loss.value if want_loss else None

    def gather_rows(self, src, rows, dst, n_scaled=0, scale=1.0):
        """dst[b] = src[rows[b]] with the first n_scaled columns times scale
        (pd_mlp_gather_rows); src, dst 2-D float32 device tensors."""
        import torch
        n_rows, n_cols = src.shape
        B = rows.numel()
        if dst.shape != (B, n_cols):
            raise ValueError("dst must be [len(rows), n_cols]")
        st = self._lib.pd_mlp_gather_rows(self._h, _ptr(src, torch.float32, n_rows * n_cols, "src"),
                                          n_rows, n_cols, _ptr(rows, torch.int32, B, "rows"), B,
                                          int(n_scaled), float(scale),
                                          _ptr(dst, torch.float32, B * n_cols, "dst"))
        if st != PD_OK:
            raise PDError(st, "pd_mlp_gather_rows failed")

    def abs_mean(self, a):
        import torch
        out = C.c_double()
        st = self._lib.pd_mlp_abs_mean(self._h, _ptr(a, torch.float32, a.numel(), "a"), a.numel(),
                                       C.byref(out))
        if st != PD_OK:
            raise PDError(st, "pd_mlp_abs_mean failed")
        return out.value

    def gradients(self, x, target):
        import torch
        B = x.numel() // self.shape[0]
        loss = C.c_double()
        g = np.empty(self.n_params, dtype=np.float32)
        st = self._lib.pd_mlp_train_step(self._h, _ptr(x, torch.float32, B * self.shape[0], "x"),
                                         _ptr(target, torch.float32, B * self.shape[3], "target"),
                                         B, 0.0, C.byref(loss), g.ctypes.data)
        if st != PD_OK:
            raise PDError(st, "pd_mlp_train_step failed")
        return g, loss.value
