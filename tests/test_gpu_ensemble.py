"""Ensembles of independent single-level members (the C1 ensemble of the
benchmark) against the fully discrete closed form.

Each member is a periodic standing wave u = a prod_d sin(m_d pi x_d), Pi = 0
with seeded modes m_d in {1, 2, 3} and amplitude a.  On a periodic grid the
semi-discrete system keeps every Fourier mode separate, so after n RK4 steps
u = A_n u_0 and Pi = B_n u_0, where (A_n, B_n) is the first column of the n-th
power of the RK4 stability polynomial at the mode's discrete symbol (the
Laplacian's and the dissipation's eigenvalues), evaluated in 40-digit
arithmetic.  The GPU result must equal it to rounding (1e-13 of the field's
size) for every member, in batched and graph mode, at the benchmark's size
(B = 512 members of 32^3, 64 steps to t = 1).
"""
import numpy as np
import pytest

import paper_2503_09629_amd as sc
from tests.test_oracle_evolve import discrete_amplitude
from workloads import ensemble_c1, standing_wave_on_spec
from workloads.data import ensemble_params

pytestmark = pytest.mark.gpu
SIGMA = 0.32


def _check(B, n, nsteps, exec):
    spec = ensemble_c1(B, n)
    ctx = sc.Context(device="cuda:0", exec=exec, sigma=SIGMA)
    ctx.build_spec(spec, block_seed=1, min_block=16, max_block=48)
    ctx.bind()
    ctx.set_initial_data_analytic(sc.SC_ID_STANDING_WAVE, (), seed=2)
    ctx.advance(nsteps)
    amp = {}
    worst = 0.0
    for b, (m, a0) in enumerate(ensemble_params(B, 2)):
        if m not in amp:
            amp[m] = discrete_amplitude(n, m, SIGMA, nsteps)
        au, ap = amp[m]
        u0 = standing_wave_on_spec(spec, 0, m, a0)[0]
        scale = np.abs(u0).max()
        eu = np.abs(ctx.read_back(b, 0, 0) - au * u0).max() / scale
        ep = np.abs(ctx.read_back(b, 0, 1) - ap * u0).max() / (scale * max(1.0, abs(ap)))
        assert eu < 1e-13 and ep < 1e-13, (b, m, eu, ep)
        worst = max(worst, eu, ep)
    assert abs(ctx.level_time(0) - nsteps * 0.25 * 2.0 / n) < 1e-14
    ctx.close()
    return worst


@pytest.mark.parametrize("exec", [sc.SC_EXEC_BATCHED, sc.SC_EXEC_GRAPH])
def test_small_ensemble_matches_closed_form(exec):
    print("96 members of 16^3, 32 steps: worst", _check(96, 16, 32, exec))


def test_benchmark_ensemble_matches_closed_form():
    print("512 members of 32^3, 64 steps: worst", _check(512, 32, 64, sc.SC_EXEC_GRAPH))
