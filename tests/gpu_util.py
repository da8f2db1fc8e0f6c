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


# Per-precision rounding of one Cholesky-index product and of the FP32/FP64
# accumulation: split BF16 represents x = hi + lo with |x - hi - lo| <=
# 2^-18 |x| and drops lo*lo (another 2^-18), so a product carries <= 3 x
# 2^-18 relative error; FP32 adds 2^-24 per accumulation step.
U_PRODUCT = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16x3": 3.0 * 2.0 ** -18}
U_ACC = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16x3": 2.0 ** -24}


def tol_chain(prec, K, stages=4):
    """Bound on max|err| / max|ref| of a quantity made by a chain of `stages`
    contractions whose longest reduction has K terms: each stage adds a
    relative error of the product rounding plus sqrt(K) accumulation steps
    (random signs); the stages add in quadrature and the largest of many
    elements stays within 5 standard deviations, so
    tol = 5 sqrt(stages) (u_product + u_acc (sqrt(K) + 1)), times 2 for the
    equal error of the FP64 oracle's different order (FP64 only)."""
    t = 5.0 * np.sqrt(stages) * (U_PRODUCT[prec] + U_ACC[prec] * (np.sqrt(K) + 1.0))
    return 2.0 * t if prec == "fp64" else t


def bar(prec, K, stages, fp64=1e-11):
    """Parity bar of a model quantity: FP64 keeps a fixed bar (only the
    rounding order differs from the oracle); FP32 and split BF16 take
    tol_chain over the longest reduction K and the number of chained
    contractions from L to the quantity."""
    return fp64 if prec == "fp64" else tol_chain(prec, K, stages)
