"""The printed constants and workloads against the text fixtures under
tests/golden/ (each row of a fixture cites where the paper prints it), and
the oracle's refusal of a non-finite indicator sum."""
import math

import numpy as np
import pytest

import workloads as W
from fixtures import paper_parameters, shock_tubes


def test_oracle_uses_the_printed_parameters(orc):
    params = paper_parameters()
    assert len(params) == 12
    for name, value in params.items():
        if name == "cfl":
            assert W.CFL == float(value)
        else:
            assert orc.param(name) == float(value), name
    assert math.isnan(orc.param("no such parameter"))


def test_shock_tube_states_are_the_printed_ones():
    tubes = shock_tubes()
    assert set(tubes) == {"sod", "lax"}
    assert (tubes["sod"]["left"], tubes["sod"]["right"]) == W.SOD
    assert (tubes["lax"]["left"], tubes["lax"]["right"]) == W.LAX


def test_gamma_sum_overflow_is_reported(orc):
    """A jump of 1e12 beside exactly constant data makes tau/(beta_k + eps)
    about 1e64, so the literal gamma_k overflows and chi_k is undefined: the
    oracle reports it (status and, for a grid, an error) instead of taking a
    decision from inf/inf."""
    v = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 1e12])
    out, tr = orc.teno_m(6, orc.LIM_MP, 1e-5, v)
    assert tr.status == orc.ENONFINITE and math.isnan(out)
    out, tr = orc.teno_m(6, orc.LIM_MP, 1e-5, v * 1e-12)
    assert tr.status == 0 and math.isfinite(out)
    grid = dict(ndim=1, n=[16], dx=[0.1], bc=[1], system=0, adv=[1.0])
    U = np.zeros((1, 16))
    U[0, 12:] = 1e12
    with pytest.raises(orc.NonFiniteIndicator):
        orc.reconstruct_faces(U, grid, 6, orc.LIM_MP, 1e-5, 1.4, 0)
    with pytest.raises(orc.NonFiniteIndicator):
        orc.rk3_step(U, grid, 6, orc.LIM_MP, 1e-5, 1.4, 1e-3)
    with pytest.raises(orc.NonFiniteIndicator):
        orc.rk3_points(U, grid, 6, orc.LIM_MP, 1e-5, 1.4, 1e-3, np.array([10]))
    # the same shape at magnitude 1 is fine
    orc.reconstruct_faces(U * 1e-12, grid, 6, orc.LIM_MP, 1e-5, 1.4, 0)
