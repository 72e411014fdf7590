"""Oracle: transient sequence with adaptive time steps (test infrastructure only).

Section 4 of the paper: a sequence of backward-Euler steps, each an EDFA-preconditioned
solve of the block system from x0 = 0, with

* the step size of eq. delta_t_dyn,
      dt_{n+1} = min( dt_n * min(dt_mult, dp_T / dp_max), dt_max ),
  dp_max the largest pressure change over the cells between the last two steps;
* the Courant number of eq. CFL_number, chi^E = Q^E dt / (Omega^E phi^E), and its maximum
  chi_inf over the cells, reported per step (its mean over the steps is the paper's
  second measure);
* stage 1 of the preconditioner built once and recycled: A_pipi, A_pip and A_ppi do not
  depend on dt or on the previous pressure, so only stage 2 is rebuilt per step
  (Section 3, implementation details); optionally stage 1 too every k steps.

Readings where the paper is silent (stated again in the design notes):
* dp_max is the largest absolute change max_E |p_n^E - p_{n-1}^E|; dp_max = 0 grows the
  step by dt_mult;
* Q^E, "the water flux through element E", is half the sum of the absolute outward face
  fluxes of E, sum_i |q_i^E| / 2 (inflow = outflow for a steady cell), with the local
  fluxes q^E = W^E (p^E 1 - pi^E) of eq. fluxes_MHFEM_3 (Dirichlet faces at their value).

Pins (tests/test_oracle_transient.py): the Courant number of a homogeneous brick grid under
a linear pressure in closed form; global mass balance of each step (storage change equals
the net boundary inflow through the Dirichlet faces); the step sequence of an unlimited
pressure goal in closed form (dt0 dt_mult^k capped at dt_max); a step on which the pressure
goal binds lands the next change near the goal; long steps reach the steady solution.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

from . import edfa as oedfa, krylov, mhfe


@dataclass
class StepParams:
    n_steps: int = 10
    dt0: float = 1e-3
    dt_mult: float = 2.0
    dt_max: float = np.inf
    dp_target: float = np.inf
    porosity: float = 0.2
    t_end: float = np.inf
    stage1_every: int = 0          # 0: stage 1 built once
    rtol: float = 1e-8
    restart: int = 50
    method: str = "gmres"          # "gmres" | "bicgstab"
    max_iter: int = 5000


@dataclass
class StepRecord:
    t: float
    dt: float
    iterations: int
    converged: bool
    dp_max: float
    chi_inf: float


@dataclass
class Sequence:
    steps: list = field(default_factory=list)
    u: np.ndarray = None           # last solution

    @property
    def chi_mean(self):
        return float(np.mean([s.chi_inf for s in self.steps])) if self.steps else 0.0


def face_values(s: mhfe.System, u, bc_value):
    """pi on every face: the unknowns, Dirichlet faces at their prescribed value."""
    pi = np.asarray(bc_value, dtype=np.float64).copy()
    pi[s.ufaces] = u[:s.nfu]
    return pi


def element_fluxes(s: mhfe.System, u, bc_value):
    """q^E = W^E (p^E 1 - pi^E) (eq. fluxes_MHFEM_3), outward, per cell and local face."""
    pi = face_values(s, u, bc_value)[s.topo.cell_faces]          # (Ne, 6)
    p = u[s.nfu:]
    return np.einsum("eab,eb->ea", s.W, p[:, None] - pi)


def chi_inf(s: mhfe.System, u, bc_value, dt, porosity):
    """max_E chi^E, chi^E = Q^E dt / (Omega^E phi) (eq. CFL_number), Q^E = sum_i |q_i^E| / 2."""
    Q = 0.5 * np.abs(element_fluxes(s, u, bc_value)).sum(axis=1)
    return float(np.max(Q * dt / (s.vol * porosity)))


def next_dt(dt, dp_max, prm: StepParams):
    """eq. delta_t_dyn."""
    grow = prm.dt_mult if dp_max <= 0.0 else min(prm.dt_mult, prm.dp_target / dp_max)
    return min(dt * grow, prm.dt_max)


def run(prob, eprm: oedfa.Params, prm: StepParams, workers=1) -> Sequence:
    """The sequence from prob.p_prev.  Returns per-step records and the last solution."""
    out = Sequence()
    p_prev = np.asarray(prob.p_prev, dtype=np.float64).copy()
    dt, t = prm.dt0, 0.0
    st1 = None
    for k in range(prm.n_steps):
        pk = dataclasses.replace(prob, dt=dt, p_prev=p_prev)
        s = mhfe.assemble(pk)
        if st1 is None or (prm.stage1_every > 0 and k % prm.stage1_every == 0):
            st1 = oedfa.stage1(s, eprm, workers=workers)
        st2 = oedfa.stage2(s, st1, eprm)
        E = oedfa.Edfa(s, eprm, st1, st2)
        A = s.matrix()
        if prm.method == "bicgstab":
            r = krylov.bicgstab(lambda v: A @ v, E.apply, s.b, prm.rtol, prm.max_iter)
        else:
            r = krylov.gmres(lambda v: A @ v, E.apply, s.b, prm.rtol, prm.restart, prm.max_iter)
        u = r.x
        p = u[s.nfu:]
        dp = float(np.max(np.abs(p - p_prev))) if p.size else 0.0
        chi = chi_inf(s, u, prob.bc_value, dt, prm.porosity)
        t += dt
        out.steps.append(StepRecord(t, dt, r.iterations, r.converged, dp, chi))
        out.u = u
        if not r.converged or t >= prm.t_end:
            break
        p_prev = p.copy()
        dt = next_dt(dt, dp, prm)
    return out
