"""Helpers shared by the GPU tests (not collected as tests)."""
import numpy as np

import pd_inputs as P
from oracle import pd as opd


def oracle_model(scene, build_schur=True):
    return opd.PDModel(scene.rest, scene.tets, scene.mu, scene.dirichlet, scene.region,
                       build_schur=build_schur)


def gpu_context(scene, **kw):
    from paper_2008_01541_amd import PDContext
    return PDContext(scene.rest, scene.tets, scene.region, scene.dirichlet, scene.mu, **kw)


def dev(a, dtype=None):
    import torch
    a = np.ascontiguousarray(a)
    t = torch.tensor(a.reshape(-1), device="cuda")
    return t if dtype is None else t.to(dtype)


def host(t, shape=None):
    a = t.detach().cpu().numpy()
    return a if shape is None else a.reshape(shape)


def rel(a, b):
    d = np.abs(np.asarray(a) - np.asarray(b)).max()
    s = max(np.abs(np.asarray(b)).max(), 1e-300)
    return d / s


SMALL_SCENES = {
    "cube8": lambda: P.scene_cube8(),
    "g4x3x5": lambda: P.scene_small(4, 3, 5, h=1.0, region_top_layers=2, seed=3),
    "g9x7x6": lambda: P.scene_small(9, 7, 6, h=0.5, region_top_layers=2, seed=4),
    "g16x15x8": lambda: P.scene_small(16, 15, 8, h=1.0, region_top_layers=2, seed=5),
    "g3x3x3_allregion": lambda: P.scene_small(3, 3, 3, h=1.0, region_top_layers=4, seed=6),
}
