"""The smoother's colour orderings against point-by-point Gauss-Seidel.

The update of eq. (19) moves one cell by its residual over the diagonal of L.
Visiting cells one at a time, each from the current field, is Gauss-Seidel by
definition; here it is written from the operator alone (L applied to the whole
field, the diagonal probed with unit fields), with none of the oracle's
colour-class code.  Four colour classes ((i + j) mod 2) + 2 ((j + k) mod 2)
give every stencil neighbour another class, so one four-class sweep equals
that sequential sweep in class order, whatever the order inside each class.
The paper's red-black does not: its in-plane edge terms join same-colour
cells, so the red-black sweep is a Jacobi step inside each colour.
"""
import numpy as np
import pytest

from oracle import mg, ref

STENCIL = [(a, b, 0) for a in (-1, 0, 1) for b in (-1, 0, 1) if (a, b) != (0, 0)] + \
          [(a, 0, c) for a in (-1, 0, 1) for c in (-1, 1)] + [(0, b, c) for b in (-1, 1) for c in (-1, 1)]


def _problem(shape=(4, 4, 6), seed=0, lam_dt_h2=3.0):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((3,) + shape)
    S = rng.standard_normal((3,) + shape)
    eta = np.exp(rng.uniform(-1.5, 1.5, shape))
    h = 0.1
    return B, S, eta, h, lam_dt_h2 * h * h


def _diag(eta, h, lam_dt):
    """diag[c, k, j, i] = (L e)_c at (i, j, k) for the unit field e at that
    component and cell."""
    d = np.empty((3,) + eta.shape)
    for c in range(3):
        for p in np.ndindex(eta.shape):
            e = np.zeros((3,) + eta.shape)
            e[(c,) + p] = 1.0
            d[(c,) + p] = ref.apply(e, eta, h, lam_dt)[(c,) + p]
    return d


def _sequential_gs(B, S, eta, h, lam_dt, cells):
    """Gauss-Seidel over `cells` (list of (k, j, i)) in the given order: each
    component of each cell moves by (S - L B) / diag from the current B."""
    B = B.copy()
    d = _diag(eta, h, lam_dt)
    for p in cells:
        for c in range(3):
            r = S[(c,) + p] - ref.apply(B, eta, h, lam_dt)[(c,) + p]
            B[(c,) + p] += r / d[(c,) + p]
    return B


def _class_order(shape, classes, ncls, rng):
    cells = []
    for m in range(ncls):
        sel = [p for p in np.ndindex(shape) if classes[p] == m]
        cells += [sel[i] for i in rng.permutation(len(sel))]
    return cells


def test_four_classes_separate_every_stencil_neighbour():
    """On an even periodic grid every one of the 18 stencil offsets (6 faces,
    12 in-plane edges) leads to another class under the four-class ordering;
    under red-black the 6 faces change colour and the 12 edges do not."""
    shape = (6, 4, 8)
    c4 = ref.colour_classes(shape, 1)
    c2 = ref.colour_classes(shape, 0)
    assert set(np.unique(c4)) == {0, 1, 2, 3} and set(np.unique(c2)) == {0, 1}
    assert len(STENCIL) == 18
    for (a, b, c) in STENCIL:
        moved4 = np.roll(c4, (-c, -b, -a), axis=(0, 1, 2))
        moved2 = np.roll(c2, (-c, -b, -a), axis=(0, 1, 2))
        assert (moved4 != c4).all(), (a, b, c)
        faces = abs(a) + abs(b) + abs(c) == 1
        assert ((moved2 != c2).all() if faces else (moved2 == c2).all()), (a, b, c)


def test_diagonal_probe_matches_alpha():
    """The probed diagonal of L is 1 + alpha_c of eqs. (21)-(23): the pivot the
    sequential reference divides by is the smoother's."""
    _, _, eta, h, lam_dt = _problem()
    assert np.allclose(_diag(eta, h, lam_dt), 1.0 + ref.alpha(eta, h, lam_dt), rtol=1e-14, atol=0)


@pytest.mark.parametrize("seed", [0, 1])
def test_four_class_sweep_is_sequential_gauss_seidel(seed):
    """One four-class sweep equals Gauss-Seidel visiting the cells class by
    class in a random order inside each class (two sweeps likewise)."""
    B, S, eta, h, lam_dt = _problem(seed=seed)
    rng = np.random.default_rng(100 + seed)
    classes = ref.colour_classes(eta.shape, 1)
    scale = np.abs(B).max() + np.abs(S).max()
    seq = B
    for ns in (1, 2):
        seq = _sequential_gs(seq, S, eta, h, lam_dt, _class_order(eta.shape, classes, 4, rng))
        got = ref.smooth(B, S, eta, h, lam_dt, ns, ordering=1)
        assert np.abs(got - seq).max() <= 1e-13 * scale, ns


def test_red_black_is_a_jacobi_step_inside_each_colour():
    """The same sequential reference in red-then-black order differs from the
    red-black sweep by far more than rounding: the in-plane edge terms join
    same-colour cells, so the pin above holds for the four-class ordering only."""
    B, S, eta, h, lam_dt = _problem()
    rng = np.random.default_rng(7)
    cells = _class_order(eta.shape, ref.colour_classes(eta.shape, 0), 2, rng)
    seq = _sequential_gs(B, S, eta, h, lam_dt, cells)
    rb = ref.smooth(B, S, eta, h, lam_dt, 1)
    assert np.abs(seq - rb).max() >= 1e-3 * np.abs(rb).max()


def test_four_class_sweeps_fix_and_reach_the_solution():
    """The exact solution of L B = S is a fixed point of a four-class sweep,
    and repeated sweeps converge to it (Gauss-Seidel on this operator)."""
    B, S, eta, h, lam_dt = _problem(shape=(4, 6, 8), seed=3, lam_dt_h2=1.0)
    X = mg.direct_solve(eta, h, lam_dt, S)
    assert np.abs(ref.smooth(X, S, eta, h, lam_dt, 1, ordering=1) - X).max() <= 1e-12 * np.abs(X).max()
    errs = []
    Y = B
    for _ in range(4):
        Y = ref.smooth(Y, S, eta, h, lam_dt, 10, ordering=1)
        errs.append(np.abs(Y - X).max())
    assert all(errs[i + 1] < 0.5 * errs[i] for i in range(3)), errs
    assert errs[-1] <= 1e-3 * np.abs(B - X).max()
