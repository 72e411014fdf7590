"""Transient sequence on distorted channelised grids (the 128x128x64 workload's structure at a
size the oracle handles): dt doubles from 1e-3 each step, p_n is the previous step's
pressure, and the preconditioner is refreshed by edfa_update_dt + stage 2 only.  Stage 1
uses A_pipi, A_ppi and A_pip, which do not depend on dt (Section 3, implementation
details), so the refreshed preconditioner equals a full rebuild; each step is compared with
the oracle's full assembly, EDFA and GMRES at that dt."""
import dataclasses

import numpy as np
import pytest

from oracle import edfa as oedfa, krylov, mhfe
from paper_2009_13916_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("full_resetup", [False, True])
def test_transient_sequence_matches_oracle(lib, full_resetup):
    import torch
    prob = inputs.channel_problem(8, 7, 4, contrast=1e6, perturb=0.2, config_id=81, dt=1e-3)
    kw = dict(variant="dynamic", n_add=1, n_ent=6, tau=1e-3, filt="post_H")
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**kw))
    p_prev = np.asarray(prob.p_prev, dtype=np.float64).copy()
    for k in range(4):
        dt = 1e-3 * 2.0 ** k
        if k > 0:
            S.update_dt(dt, torch.tensor(p_prev, device="cuda"))
            if full_resetup:
                P.resetup()
            else:
                P.stage2()
        x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-8, restart=50)
        pk = dataclasses.replace(prob, dt=dt, p_prev=p_prev.copy())
        o = mhfe.assemble(pk)
        A = o.matrix()
        E = oedfa.build(o, oedfa.Params(**kw))
        ref = krylov.gmres(lambda v: A @ v, E.apply, o.b, 1e-8, 50)
        xg = x.cpu().numpy()
        assert st == 0
        assert np.linalg.norm(o.b - A @ xg) <= 1e-8 * np.linalg.norm(o.b), k
        dp = np.linalg.norm(xg[o.nfu:] - ref.x[o.nfu:]) / np.linalg.norm(ref.x[o.nfu:])
        print(f"[transient] step {k} dt {dt:.0e}: {info['iterations']} iterations "
              f"(oracle {ref.iterations}), pressure vs oracle {dp:.2e}", flush=True)
        assert dp <= 1e-8, (k, dp)
        assert abs(info["iterations"] - ref.iterations) <= 2, (k, info["iterations"], ref.iterations)
        p_prev = xg[o.nfu:].copy()


ADAPT = dict(variant="dynamic", n_add=1, n_ent=6, tau=1e-3, filt="post_H")


def _adaptive_problem():
    """Distorted channel grid with a storage coefficient large enough for a real transient."""
    prob = inputs.channel_problem(7, 6, 4, contrast=1e3, perturb=0.2, config_id=82, dt=1e-3)
    return dataclasses.replace(prob, c=np.full(prob.n_cells, 0.2))


@pytest.mark.parametrize("method", ["gmres", "bicgstab"])
def test_adaptive_sequence_matches_oracle(lib, method):
    """edfa_transient against the oracle sequence: per step the same dt (eq. delta_t_dyn with
    the pressure goal binding on some steps), pressure to 1e-8, iterations +-2, dp_max and
    chi_inf to 1e-7."""
    from oracle import transient as otr
    prob = _adaptive_problem()
    sp = otr.StepParams(n_steps=7, dt0=1e-3, dt_mult=3.0, dt_max=0.5, dp_target=0.08,
                        porosity=0.2, method=method, max_iter=2000)
    ref = otr.run(prob, oedfa.Params(**ADAPT), sp)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**ADAPT))
    u, steps, st = lib.transient(S, P, n_steps=7, dt0=1e-3, dt_mult=3.0, dt_max=0.5,
                                 dp_target=0.08, porosity=0.2, method=method, max_iter=2000)
    assert st == 0 and len(steps) == len(ref.steps) == 7
    limited = 0
    for k, (g, o) in enumerate(zip(steps, ref.steps)):
        print(f"[transient adaptive {method}] step {k}: dt {g['dt']:.4e} (oracle {o.dt:.4e}), "
              f"iterations {g['iterations']} ({o.iterations}), dp {g['dp_max']:.3e}, "
              f"chi {g['chi_inf']:.3e}", flush=True)
        assert g["dt"] == pytest.approx(o.dt, rel=1e-7)
        assert g["t"] == pytest.approx(o.t, rel=1e-7)
        assert g["converged"] == 1
        assert abs(g["iterations"] - o.iterations) <= 2
        assert g["dp_max"] == pytest.approx(o.dp_max, rel=1e-7)
        assert g["chi_inf"] == pytest.approx(o.chi_inf, rel=1e-7)
        limited += sp.dp_target / o.dp_max < sp.dt_mult
    assert limited >= 1
    nfu = S.info["nfu"]
    p, pr = u.cpu().numpy()[nfu:], ref.u[nfu:]
    assert np.linalg.norm(p - pr) <= 1e-8 * np.linalg.norm(pr)


def test_adaptive_sequence_stage1_rebuilds_and_end_time(lib):
    """stage1_every = 2 gives the same sequence (stage 1 does not depend on dt); t_end stops
    the sequence at the step that reaches it."""
    prob = _adaptive_problem()
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**ADAPT))
    u1, s1, st1 = lib.transient(S, P, n_steps=5, dt0=1e-3, dt_mult=3.0, dp_target=0.08)
    S2 = lib.System(prob)
    P2 = lib.Precond(S2, lib.Params(**ADAPT))
    u2, s2, st2 = lib.transient(S2, P2, n_steps=5, dt0=1e-3, dt_mult=3.0, dp_target=0.08,
                                stage1_every=2)
    assert st1 == st2 == 0
    assert [a["dt"] for a in s1] == pytest.approx([b["dt"] for b in s2], rel=1e-12)
    assert torch_allclose(u1, u2)
    S3 = lib.System(prob)
    P3 = lib.Precond(S3, lib.Params(**ADAPT))
    t_end = s1[2]["t"] * (1 - 1e-9)
    u3, s3, st3 = lib.transient(S3, P3, n_steps=5, dt0=1e-3, dt_mult=3.0, dp_target=0.08,
                                t_end=t_end)
    assert len(s3) == 3 and s3[-1]["t"] >= t_end


def torch_allclose(a, b):
    return float((a - b).norm() / b.norm()) <= 1e-10
