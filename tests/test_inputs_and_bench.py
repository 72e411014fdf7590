"""Host logic: the seeded input generators keep the recipe they promise (determinism, shapes,
the statistics of the random fields, the channel fraction, the batch draws), and bench.py's
helpers (algorithmic bytes, the PMC traffic record, the one-GPU rule)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2009_13916_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_generators_are_deterministic():
    a = inputs.full_tensor_problem(6, sigma=2.0, corr=2.0, config_id=7)
    b = inputs.full_tensor_problem(6, sigma=2.0, corr=2.0, config_id=7)
    c = inputs.full_tensor_problem(6, sigma=2.0, corr=2.0, config_id=8)
    assert np.array_equal(a.K, b.K) and np.array_equal(a.p_prev, b.p_prev)
    assert not np.array_equal(a.K, c.K)


def test_problem_shapes_and_boundary_codes():
    p = inputs.channel_problem(6, 5, 4, contrast=1e6, config_id=3)
    ne, nf = p.n_cells, p.n_faces
    assert p.nodes.shape == (7 * 6 * 5, 3) and p.K.shape == (ne, 6)
    assert p.bc_type.shape == (nf,) and p.bc_value.shape == (nf,)
    # Dirichlet exactly on the x = 0 and x = 1 faces: p = 1 and 0
    nxf = 7 * 5 * 4
    xf = np.arange(nxf)
    i = xf % 7
    assert np.all(p.bc_type[:nxf][(i == 0) | (i == 6)] == inputs.BC_DIRICHLET)
    assert np.all(p.bc_type[:nxf][(i > 0) & (i < 6)] == inputs.BC_NEUMANN)
    assert np.all(p.bc_type[nxf:] == inputs.BC_NEUMANN)
    assert np.all(p.bc_value[:nxf][i == 0] == 1.0) and np.all(p.bc_value[:nxf][i == 6] == 0.0)


def test_distorted_nodes_stay_inside_their_cells():
    p = inputs.channel_problem(8, 8, 4, perturb=0.2, config_id=3)
    X = p.nodes.reshape(5, 9, 9, 3)          # k, j, i
    ref = inputs.brick_nodes(8, 8, 4).reshape(5, 9, 9, 3)
    d = np.abs(X - ref)
    assert d[..., 0].max() <= 0.2 / 8 + 1e-15 and d[..., 2].max() <= 0.2 / 4 + 1e-15
    # boundary nodes fixed
    assert np.array_equal(X[0], ref[0]) and np.array_equal(X[:, :, 0], ref[:, :, 0])


def test_full_tensor_permeability_recipe():
    p = inputs.full_tensor_problem(16, sigma=2.0, corr=4.0, config_id=2)
    K = np.zeros((p.n_cells, 3, 3))
    idx = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (0, 2): 4, (1, 2): 5}
    for (a, b), c in idx.items():
        K[:, a, b] = K[:, b, a] = p.K[:, c]
    ev = np.linalg.eigvalsh(K)               # ascending: k1/a, k1/sqrt(a), k1
    ratio = ev[:, 2] / ev[:, 0]
    assert np.all(ev > 0)
    assert ratio.min() >= 10 * (1 - 1e-9) and ratio.max() <= 100 * (1 + 1e-9)
    assert np.allclose(ev[:, 1] ** 2, ev[:, 0] * ev[:, 2], rtol=1e-9)
    lnk1 = np.log(ev[:, 2])
    assert abs(lnk1.std() - 2.0) < 1e-9      # standardised, then scaled to sigma


def test_channel_fraction_and_contrast():
    p = inputs.channel_problem(32, 32, 16, contrast=1e6, config_id=3)
    k = p.K[:, 0]
    assert set(np.unique(k)) == {1.0, 1e-6}
    assert (k == 1.0).mean() >= 0.30


def test_haar_rotations_are_rotations():
    R = inputs.haar_rotations(200, np.random.default_rng(0))
    assert np.allclose(np.einsum("nij,nkj->nik", R, R), np.eye(3)[None], atol=1e-12)
    assert np.allclose(np.linalg.det(R), 1.0)


def test_batch_draws():
    probs = inputs.batch_problems(64, 8, 32)
    sides = np.array([p.nx for p in probs])
    assert sides.min() >= 8 and sides.max() <= 32 and len(set(sides)) > 10
    assert all(p.nx == p.ny == p.nz for p in probs)


def test_observations_unique():
    cells, target = inputs.observations(1000, 64, np.random.default_rng(1))
    assert len(np.unique(cells)) == 64 and np.all((target >= 0) & (target <= 1))


def test_bench_helpers(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    assert bench.spmv_bytes(10, 4) == 12 * 10 + 4 * 5 + 8 * 4 + 8 * 4
    r = {"value_bytes": 8, "nnz": 10, "rows": 4, "cols": 4}
    assert bench.slot_bytes(r) == bench.spmv_bytes(10, 4)
    assert bench.kernel_label("chunk/12", "M_L", 1).startswith("k_spmv_chunk<double, double, 12>")
    assert bench.kernel_label("sell/4", "G_F", 1).startswith("k_spmv_sell<double, double, 1, 4>")
    # per-kernel totals of a profiled solve: two matrices on one kernel are summed
    info = {"slot_ms": {"M_L": 0.04, "M_U": 0.04, "G_F": 0.016},
            "slot_launches": {"M_L": 10, "M_U": 10, "G_F": 20}}
    rep = {k: {"variant": v, "value_bytes": 8, "nnz": 1000, "rows": 100, "cols": 100}
           for k, v in (("M_L", "chunk/12"), ("M_U", "chunk/12"), ("G_F", "sell/4"))}
    fam, kern = bench.families(info, rep, 10)
    k = kern["k_spmv_chunk<double, double, 12>"]
    assert k["launches"] == 20 and abs(k["ms"] - 0.8) < 1e-12 and k["matrices"] == ["M_L", "M_U"]
    assert {f["matrix"] for f in fam} == {"M_L", "M_U", "G_F"}
    # a kernel's traffic is the launch-weighted mean of its matrices' measured bytes, read
    # only for the kernel source it was taken on and only when every matrix is covered
    chunk, sell = "k_spmv_chunk<double, double, 12>", "k_spmv_sell<double, double, 1, 4>"
    rec = {"kernel_sha": bench.spmv_kernel_sha(),
           "matrices": {"M_L": {"kernel": chunk, "hbm_bytes_per_launch": 100.0},
                        "M_U": {"kernel": chunk, "hbm_bytes_per_launch": 300.0}}}
    path = tmp_path / "traffic.md"

    def write(r):
        path.write_text("# traffic\n\n```json\n" + json.dumps(r) + "\n```\n")
    old = bench.TRAFFIC
    bench.TRAFFIC = str(path)
    try:
        write(rec)
        fam[[f["matrix"] for f in fam].index("M_U")]["launches"] = 30
        assert bench.measured_traffic(chunk, fam) == (100.0 * 10 + 300.0 * 30) / 40
        assert bench.measured_traffic(sell, fam) is None          # G_F not measured
        rec["matrices"]["M_U"]["kernel"] = sell                   # measured on another kernel
        write(rec)
        assert bench.measured_traffic(chunk, fam) is None
        rec["matrices"]["M_U"]["kernel"] = chunk
        rec["kernel_sha"] = "0" * 16                              # another kernel source
        write(rec)
        assert bench.measured_traffic(chunk, fam) is None
    finally:
        bench.TRAFFIC = old
    # the committed record, when present, parses and names its matrices' kernels
    if os.path.exists(bench.TRAFFIC):
        rec = json.loads(open(bench.TRAFFIC).read().split("```json")[1].split("```")[0])
        assert all("kernel" in m and m["hbm_bytes_per_launch"] > 0
                   for m in rec["matrices"].values())


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
