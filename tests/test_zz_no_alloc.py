"""sc_norms_noalloc, the reduction entry point for callers that cannot
allocate device memory, against sc_norms: the same reduction shape, so the
results must be equal bit for bit.  Two calls in a row, the second on a
smaller level, since the static workspace keeps the previous call's partials.
"""
import numpy as np
import pytest

import paper_2503_09629_amd as sc
from workloads import config_c3, pulses_on_spec

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [sc.SC_FP64, sc.SC_MIXED])
def test_noalloc_norms_equal_arena_norms(precision):
    spec = config_c3(64, nlev=3)
    ctx = sc.Context(device="cuda:0", precision=precision)
    ctx.build_spec(spec)
    ctx.bind()
    for l in range(spec.nlevels):
        for v, f in enumerate(pulses_on_spec(spec, l)):
            ctx.set_initial_data(0, l, v, f)
    ctx.advance(2)
    sizes = [ctx.counts(l)[1] for l in range(spec.nlevels)]
    big = int(np.argmax(sizes))
    small = int(np.argmin(sizes))
    assert sizes[small] < sizes[big]
    for level, var, arr in ((big, 1, sc.SC_ARR_Y), (small, 0, sc.SC_ARR_Y),
                            (big, 0, sc.SC_ARR_K2), (small, 1, sc.SC_ARR_K1)):
        want = ctx.norms(0, level, var, arr)
        got = ctx.norms_noalloc(0, level, var, arr)
        assert np.array_equal(got, want), (level, var, arr, got, want)
        assert want[0] > 0 and want[2] == 0
    ctx.close()
