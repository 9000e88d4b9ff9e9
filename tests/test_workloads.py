"""Workload generators: the fast per-step C4 values equal a rebuilt matrix."""
import numpy as np

from workloads import configs


def test_c4_step_values_equal_rebuilt_matrix():
    A1, _ = configs.c4_matrix(1, 48, 40)
    kinds = configs.c4_kinds(A1, 48)
    for step in (1, 2, 77, 150, 300):
        A, th = configs.c4_matrix(step, 48, 40)
        v, th2 = configs.c4_step_values(step, kinds, 48)
        assert np.array_equal(A.col, A1.col) and np.array_equal(A.row_ptr, A1.row_ptr)
        assert np.array_equal(v, A.val) and th == th2
