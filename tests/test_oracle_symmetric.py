"""Pins for the symmetric NN coupling (the remark after Sec. 3.2): the coupling of Sec. 3.2
unchanged on the cell-centred points x_i = (i + 1/2) h, so that each coarse point is the centre
of its 2 x 2 block of fine points.  Only where the data and test functions are sampled changes;
the oracle evaluates them at the shifted points directly.  Checked against closed forms that
do not use the oracle: the field samples, the exact mean of a linear observable (every N), and
at high density E[P_l] = S_l and the linear pair variance.  Tolerances 4.5 standard errors."""
import math

import numpy as np
import pytest

import dk_workloads as W
import oracle
from closed_forms import field_np, fluct_second_moment, linear_mean, pair_variance_linear

Z = 4.5


@pytest.mark.parametrize("make", [W.config1, W.config3, lambda: W.paper_irreg()])
def test_fields_at_cell_centres(make):
    p = make()
    for f in [p.rho0] + [o.phi for o in p.obs]:
        for n in (8, 12, 32):
            a = oracle.field_grid(f, p.box, n, 0.5)
            b = field_np(f, p.box, n, 0.5)
            assert np.max(np.abs(a - b)) <= 1e-13 * max(1.0, np.max(np.abs(b)))
    # and the grid really moved: a mode that vanishes at the vertices does not at the centres
    m = W.Field(W.FIELD_MODES, 0.0, [W.sin_mode(2, 0)])
    assert np.max(np.abs(oracle.field_grid(m, 1.0, 4, 0.0))) < 1e-15
    assert np.min(np.abs(oracle.field_grid(m, 1.0, 4, 0.5))) > 0.99


def test_exact_linear_mean_on_cell_centres():
    p = W.config1().with_(grid=W.GRID_CELL)
    op = oracle.OracleProblem(p)
    X = oracle.run_range(op, 0, 0, 2000, tag=W.TAG_MC)[:, 0, 0]
    ref = linear_mean(p, 0, p.obs[0].phi)
    assert abs(X.mean() - ref) < Z * X.std(ddof=1) / math.sqrt(len(X))


@pytest.mark.parametrize("level", [0, 1, 2])
def test_square_observable_mean_high_density_cell_centres(level):
    p = W.paper_reg(N=2e9).with_(grid=W.GRID_CELL)
    P = oracle.run_range(oracle.OracleProblem(p), level, 0, 3000, coupled=False)[:, 0, 0]
    S = fluct_second_moment(p, level, p.obs[0].phi)
    assert abs(P.mean() - S) < Z * P.std(ddof=1) / math.sqrt(len(P))


@pytest.mark.parametrize("level,count", [(1, 3000), (2, 1500)])
def test_symmetric_pair_variance_linear(level, count):
    base = W.paper_reg(N=2e9).with_(grid=W.GRID_CELL)
    phi = base.obs[0].phi
    p = base.with_(obs=[W.Obs(phi, True, True, W.PSI_ID)])
    P = oracle.run_range(oracle.OracleProblem(p), level, 0, count)
    Y = P[:, 0, 0] - P[:, 0, 1]
    V = pair_variance_linear(p, level, phi)
    assert abs(Y.mean()) < Z * Y.std(ddof=1) / math.sqrt(len(Y))
    assert abs(Y.var(ddof=1) / V - 1.0) < Z * math.sqrt(2.0 / len(Y)), (Y.var(ddof=1), V)
