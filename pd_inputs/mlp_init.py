"""Seeded initial parameters of the warm-start network (an input of both the
GPU path and the oracle): He-uniform weights, zero biases."""
import numpy as np


def mlp_init_params(n_in, n_h1, n_h2, n_out, seed, out_scale=0.1):
    rng = np.random.default_rng(seed)

    def lin(fan_out, fan_in):
        lim = np.sqrt(6.0 / fan_in)
        return rng.uniform(-lim, lim, size=(fan_out, fan_in))

    return {"W1": lin(n_h1, n_in), "b1": np.zeros(n_h1),
            "W2": lin(n_h2, n_h1), "b2": np.zeros(n_h2),
            "W3": lin(n_out, n_h2) * out_scale, "b3": np.zeros(n_out)}


PARAM_ORDER = ["W1", "b1", "W2", "b2", "W3", "b3"]


def pack(params):
    return np.concatenate([np.asarray(params[k], dtype=np.float32).reshape(-1) for k in PARAM_ORDER])


def unpack(flat, n_in, n_h1, n_h2, n_out):
    shapes = {"W1": (n_h1, n_in), "b1": (n_h1,), "W2": (n_h2, n_h1), "b2": (n_h2,),
              "W3": (n_out, n_h2), "b3": (n_out,)}
    out, o = {}, 0
    for k in PARAM_ORDER:
        n = int(np.prod(shapes[k]))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shapes[k])
        o += n
    return out
