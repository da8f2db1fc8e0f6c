"""Pins of the sampled oracle (oracle/sampled.py: the MLCC2 quantities at
sampled elements, for workloads too large for the host) against the dense
oracle on small problems, with singles amplitudes and trial vectors of small
support and dense ones (CPU only)."""
import numpy as np
import pytest

from oracle import mlcc as om
from oracle import sampled as sm
from paper_2006_05226_amd.synth import gen_inputs

pytestmark = pytest.mark.filterwarnings("ignore::numpy.exceptions.ComplexWarning")

O, V, J, o, v = 6, 16, 24, 3, 7


def setup(seed=3):
    inp = gen_inputs(O, V, J, o, v, seed=seed)
    return inp, om.Dims(O, V, o, v), sm.DenseSource(inp.L)


def sparse_singles(seed, rows, cols, scale):
    rng = np.random.default_rng(seed)
    t = np.zeros((V, O))
    t[np.ix_(rows, cols)] = scale * rng.standard_normal((len(rows), len(cols)))
    return t


# support across active and inactive virtual / occupied orbitals
T_SPARSE = dict(rows=[0, 2, 9, 13], cols=[1, 4])
C_SPARSE = dict(rows=[1, 5, 11], cols=[0, 2, 5])


def amplitudes(kind):
    if kind == "sparse":
        return sparse_singles(7, scale=0.05, **T_SPARSE)
    return 0.05 * np.random.default_rng(8).standard_normal((V, O))


@pytest.mark.parametrize("kind", ["sparse", "dense"])
def test_lt_and_fock_blocks(kind):
    inp, d, src = setup()
    t1 = amplitudes(kind)
    D = om.dress(inp.L, inp.eps, d, t1)
    rows, cols = np.array([0, 3, 7, 12, 21]), np.array([5, 1, 8, 19])
    lt = sm.lt_block(src, t1, d, np.arange(J), rows, cols)
    assert np.abs(lt - D.Lt[np.ix_(np.arange(J), rows, cols)]).max() < 1e-15
    F = sm.fock_block(src, inp.eps, d, t1, rows, cols)
    assert np.abs(F - D.Ft[np.ix_(rows, cols)]).max() < 1e-14


@pytest.mark.parametrize("kind", ["sparse", "dense"])
def test_g_and_omega_samples(kind):
    inp, d, src = setup()
    t1 = amplitudes(kind)
    P = om.Problem(inp.L, inp.eps, d, "mlcc2")
    s = P.s_analytic(t1)
    ref1, _ = P.omega(t1, s)
    g = om.g_aibj(om.dress(inp.L, inp.eps, d, t1).Lt, d)
    quads = [(a, i, b, j) for a in range(v) for i in range(o) for b in range(v) for j in range(o)]
    got = sm.g_samples(src, t1, d, quads)
    assert np.abs(got - g.ravel()).max() < 1e-15 * max(1.0, np.abs(g).max()) * 10
    pairs = [(A, I) for A in range(V) for I in range(O)]
    om1 = sm.omega1_samples(src, inp.eps, d, t1, pairs)
    assert np.abs(om1 - ref1.ravel()).max() < 1e-14 * np.abs(ref1).max()


@pytest.mark.parametrize("kind", ["sparse", "dense"])
def test_effective_sigma_samples(kind):
    """A11 c + A12 (w - eps)^-1 A21 c from the dense complex-step Jacobian."""
    inp, d, src = setup()
    t1 = amplitudes(kind)
    P = om.Problem(inp.L, inp.eps, d, "mlcc2")
    s = P.s_analytic(t1)
    c1 = sparse_singles(9, scale=1.0, **C_SPARSE) if kind == "sparse" else \
        np.random.default_rng(10).standard_normal((V, O))
    w = 0.37
    _, a21 = om.jacobian_transform(P, t1, s, c1, np.zeros((v, o, v, o)))
    r1, _ = om.jacobian_transform(P, t1, s, c1, a21 / (w - om.orbital_denominators(inp.eps, d)))
    pairs = [(A, I) for A in range(V) for I in range(O)]
    got = sm.eff_sigma_samples(src, inp.eps, d, t1, c1, w, pairs)
    assert np.abs(got - r1.ravel()).max() < 1e-12 * np.abs(r1).max()


def test_planted_mistakes_fail(monkeypatch):
    inp, d, src = setup()
    t1 = amplitudes("sparse")
    P = om.Problem(inp.L, inp.eps, d, "mlcc2")
    ref1, _ = P.omega(t1, P.s_analytic(t1))
    pairs = [(A, I) for A in range(V) for I in range(O)]
    # the doubles enter: a perturbed s moves Omega
    bad = sm.omega1_samples(src, inp.eps, d, t1, pairs, s_rule=lambda g, den: -1.01 * g / den)
    assert np.abs(bad - ref1.ravel()).max() > 1e-6 * np.abs(ref1).max()
    # the X1 transform without its t L t term
    good_lt = sm.lt_block

    def lt_no_ttt(Lsrc, t, dd, Ks, rows, cols):
        full = good_lt(Lsrc, t, dd, Ks, rows, cols)
        SA, SI = sm._support(t)
        rows, cols = np.asarray(rows), np.asarray(cols)
        TAq = np.zeros((len(SA), len(cols)), dtype=t.dtype)
        TAq[:, cols < dd.O] = t[np.ix_(SA, cols[cols < dd.O])]
        TpI = np.zeros((len(rows), len(SI)), dtype=t.dtype)
        TpI[rows >= dd.O, :] = t[np.ix_(rows[rows >= dd.O] - dd.O, SI)]
        return full + np.einsum("pi,Kia,aq->Kpq", TpI, Lsrc(Ks, SI, dd.O + SA), TAq)

    monkeypatch.setattr(sm, "lt_block", lt_no_ttt)
    bad = sm.omega1_samples(src, inp.eps, d, t1, pairs)
    assert np.abs(bad - ref1.ravel()).max() > 1e-8 * np.abs(ref1).max()
