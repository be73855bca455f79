"""The direct int64-offset mesh generator writes the same CSR as the general
grid generator (every grid edge kept, same diagonal and weight draws)."""
import numpy as np
import pytest

import graphgen


@pytest.mark.parametrize("rows,cols,diag", [(2, 2, 1.0), (7, 9, 0.3), (64, 64, 0.01), (50, 31, 0.5),
                                            (300, 200, 0.01), (3, 1000, 0.2)])
def test_mesh64_equals_grid(rows, cols, diag):
    a = graphgen.mesh64(rows, cols, 1000, 5, diag)
    b = graphgen.grid(rows, cols, 1000, 5, 0.0, diag)
    assert a.n == b.n == rows * cols
    assert a.row_ptr.dtype == np.int64
    assert np.array_equal(a.row_ptr, b.row_ptr.astype(np.int64))
    assert np.array_equal(a.col, b.col)
    assert np.array_equal(a.w, b.w)


def test_mesh64_arrays_outlive_the_generator_call():
    import gc
    g = graphgen.mesh64(40, 50, 100, 3, 0.1)
    col = g.col
    ref = col.copy()
    del g
    gc.collect()
    _ = graphgen.mesh64(40, 50, 100, 4, 0.1)   # reuses freed memory if the view were dangling
    assert np.array_equal(col, ref)
