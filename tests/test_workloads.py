"""Workload generators: the fast per-step C4 values equal a rebuilt matrix;
the general sparse generator follows its recipe."""
import numpy as np
import scipy.sparse as sp

from workloads import configs, pde


def test_c4_step_values_equal_rebuilt_matrix():
    A1, _ = configs.c4_matrix(1, 48, 40)
    kinds = configs.c4_kinds(A1, 48)
    for step in (1, 2, 77, 150, 300):
        A, th = configs.c4_matrix(step, 48, 40)
        v, th2 = configs.c4_step_values(step, kinds, 48)
        assert np.array_equal(A.col, A1.col) and np.array_equal(A.row_ptr, A1.row_ptr)
        assert np.array_equal(v, A.val) and th == th2


def test_random_geometric_recipe():
    """The general sparse generator: nonpositive off-diagonals, diagonal at
    least the larger of the absolute row and column sums plus the margin,
    lognormal coupling magnitudes when asked for, and unchanged draws for
    the default form."""
    A = pde.random_geometric(3000, 8, 4, sigma=1.0, margin=0.02, margin_rand=0.02)
    S = A.scipy().tocsr()
    D = S.diagonal()
    O = S - sp.diags(D)
    assert O.max() <= 0.0
    rs = np.asarray(abs(O).sum(axis=1)).ravel()
    cs = np.asarray(abs(O).sum(axis=0)).ravel()
    slack = D - np.maximum(rs, cs)
    assert slack.min() >= 0.02 and slack.max() <= 0.04
    mags = -O.data[O.data < 0]
    assert abs(np.mean(np.log(mags))) < 0.05 and abs(np.std(np.log(mags)) - 1.0) < 0.05
    B = pde.random_geometric(500, 8, 5)
    C = pde.random_geometric(500, 8, 5, margin=0.5, margin_rand=1.0)
    assert np.array_equal(B.val, C.val) and np.array_equal(B.col, C.col)
    offd = -B.scipy().tocsr().data[B.scipy().tocsr().data < 0]
    assert offd.min() >= 0.5 and offd.max() < 1.5
