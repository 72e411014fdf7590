"""Pins for the transient oracle (eq. delta_t_dyn, eq. CFL_number): closed forms, global mass
balance, and the steady limit."""
import dataclasses

import numpy as np
import pytest

from oracle import edfa as oedfa, mhfe, transient
from paper_2009_13916_amd import inputs

DYN = oedfa.Params("dynamic", n_add=1, n_ent=4)


def _transient_problem(n=5, c=0.05, config_id=61):
    """Isotropic lognormal bricks with a storage coefficient large enough for a real
    transient (p_prev ~ U(0,1), Dirichlet 1 / 0 on x)."""
    p = inputs.lognormal_iso_problem(n, sigma=1.0, config_id=config_id)
    return dataclasses.replace(p, c=np.full(p.n_cells, c))


def test_courant_number_closed_form_linear_pressure():
    """Homogeneous k, steady linear pressure p = 1 - x on an n^3 brick grid: every x-face
    carries q = k h^2 / gamma, so Q^E = k h^2, and chi^E = k dt / (gamma h phi) in every
    cell.  A wrong Q (full instead of half the absolute sum, a dropped face, volume instead
    of area) changes the value."""
    n, k, dt, phi = 5, 3.0, 0.7, 0.25
    prob = inputs.lognormal_iso_problem(n, sigma=0.0, config_id=95)
    prob = dataclasses.replace(prob, K=inputs.iso_tensor(np.full(n ** 3, k)), c=np.zeros(n ** 3))
    s = mhfe.assemble(prob)
    u = mhfe.direct_solve(s)
    h = 1.0 / n
    assert transient.chi_inf(s, u, prob.bc_value, dt, phi) == pytest.approx(k * dt / (h * phi),
                                                                             rel=1e-12)
    q = transient.element_fluxes(s, u, prob.bc_value)
    np.testing.assert_allclose(q[:, 1], k * h * h, rtol=1e-12)      # x+ outward
    np.testing.assert_allclose(q[:, 0], -k * h * h, rtol=1e-12)     # x- inward
    np.testing.assert_allclose(q[:, 2:], 0.0, atol=1e-13 * k * h * h)


def test_each_step_conserves_mass_globally():
    """Backward Euler: sum_E Omega c (p - p_prev) / dt equals the net inflow through the
    Dirichlet faces (no-flow elsewhere, no source), with the element fluxes of the step."""
    prob = _transient_problem()
    s = mhfe.assemble(dataclasses.replace(prob, dt=0.01))
    u = mhfe.direct_solve(s)
    q = transient.element_fluxes(s, u, prob.bc_value)
    storage = np.sum(s.vol * prob.c * (u[s.nfu:] - prob.p_prev) / 0.01)
    dirichlet = s.kind[s.topo.cell_faces] == mhfe.DIRICHLET
    inflow = -np.sum(q[dirichlet])
    assert abs(storage - inflow) <= 1e-10 * max(abs(inflow), abs(storage))
    assert abs(storage) > 1e-3      # a real transient, not the steady limit


def test_step_sequence_without_pressure_goal():
    """dp_T = inf: dt_k = dt0 dt_mult^k, capped at dt_max."""
    prob = _transient_problem(4)
    prm = transient.StepParams(n_steps=6, dt0=1e-3, dt_mult=3.0, dt_max=0.05)
    seq = transient.run(prob, DYN, prm)
    dts = [st.dt for st in seq.steps]
    ref = [min(1e-3 * 3.0 ** k, 0.05) for k in range(6)]
    np.testing.assert_allclose(dts, ref, rtol=1e-15)
    np.testing.assert_allclose([st.t for st in seq.steps], np.cumsum(ref), rtol=1e-14)
    assert all(st.converged for st in seq.steps)


def test_pressure_goal_limits_the_next_change():
    """When dp_T / dp_max binds, the next step is dt dp_T / dp_max; in a relaxing transient
    the change it produces does not exceed the goal by much (the response is sublinear in dt)."""
    prob = _transient_problem(5, c=0.2)
    prm = transient.StepParams(n_steps=6, dt0=0.02, dt_mult=4.0, dp_target=0.05)
    seq = transient.run(prob, DYN, prm)
    limited = 0
    for a, b in zip(seq.steps, seq.steps[1:]):
        if prm.dp_target / a.dp_max < prm.dt_mult:
            limited += 1
            assert b.dt == pytest.approx(a.dt * prm.dp_target / a.dp_max, rel=1e-14)
            assert b.dp_max <= 1.5 * prm.dp_target
        else:
            assert b.dt == pytest.approx(a.dt * prm.dt_mult, rel=1e-14)
    assert limited >= 2


def test_long_steps_reach_the_steady_solution():
    """As dt grows the storage term vanishes: the last step's pressure is the steady one."""
    prob = _transient_problem(4, c=0.05)
    prm = transient.StepParams(n_steps=12, dt0=1e-2, dt_mult=10.0, rtol=1e-12)
    seq = transient.run(prob, DYN, prm)
    steady = mhfe.direct_solve(mhfe.assemble(dataclasses.replace(prob, c=np.zeros(prob.n_cells))))
    nfu = len(seq.u) - prob.n_cells
    assert np.linalg.norm(seq.u[nfu:] - steady[nfu:]) <= 1e-6 * np.linalg.norm(steady[nfu:])
    assert seq.steps[-1].dp_max < 1e-6
