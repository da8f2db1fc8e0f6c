"""Helpers shared by the GPU tests."""
import numpy as np

from oracle import mlcc as om
from paper_2006_05226_amd import mlcc
from paper_2006_05226_amd.synth import gen_inputs


def make(O, V, J, o, v, seed=0, model="mlcc2", precision="fp64", ctx=None):
    inp = gen_inputs(O, V, J, o, v, seed=seed)
    ctx = ctx or mlcc.Context(0)
    P = mlcc.Problem(ctx, inp.L, inp.eps, O, V, o, v, model=model, precision=precision)
    d = om.Dims(O, V, o if model != "ccs" else 0, v if model != "ccs" else 0)
    OP = om.Problem(inp.L, inp.eps, d, model)
    return inp, ctx, P, OP, d


def full_vec(c1, c2):
    parts = [c1.ravel()]
    if c2 is not None:
        parts.append(c2.ravel())
    return np.concatenate(parts)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
