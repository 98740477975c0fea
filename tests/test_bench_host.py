"""Host-side logic of bench.py (no GPU): the one-GPU contract, the lookup of
the committed HBM counter figures by kernel-source hash, and the profiler
names of the single-kernel families."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_counter_traffic_follows_the_kernel_sources_and_workload(monkeypatch, tmp_path):
    import json
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_counters.json").write_text(json.dumps(
        {"source_sha": "abc",
         "workloads": {"c3_3d96_grf": {"families": {"cheb_S_l0": {"bytes_per_launch": 1.5e8}}}}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "abc")
    assert bench.measured_traffic("c3_3d96_grf", "cheb_S_l0") == 1.5e8
    assert bench.measured_traffic("c3_3d96_grf", "no_such_family") is None
    # figures taken on another workload are not reported for this one
    assert bench.measured_traffic("c2_3d64", "cheb_S_l0") is None
    # figures taken on other kernel sources are not reported
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "def")
    assert bench.measured_traffic("c3_3d96_grf", "cheb_S_l0") is None


def test_kernel_source_hash_is_deterministic_hex():
    h = bench.kernel_source_sha()
    assert h == bench.kernel_source_sha() and len(h) == 16 and int(h, 16) >= 0


class _Shape:
    def shape(self, level):
        return (0, True)


def test_kernel_names_of_single_kernel_families():
    pc = _Shape()
    assert bench.kernel_name("cheb_S_l0", 3, pc) == "k_cheb<3, double, double, 0, true, true>"
    assert bench.kernel_name("resid_S_l0", 3, pc) == "k_lspmv<3, double, double, 0, true, true>"
    assert bench.kernel_name("spmv_K", 3, pc) == "k_spmv_K<3, double>"
    assert bench.kernel_name("spmv_K", 2, pc, flux=True) == "k_spmv_K1<2, double>"
    assert bench.kernel_name("schur_rhs", 3, pc) == "k_schur_rhs<3, double, double, false>"
    assert bench.kernel_name("schur_vel", 3, pc, flux=True) == "k_schur_vel<3, double, double, true>"
    assert bench.kernel_name("spmv_K", 3, pc, dg=True) == "k_dg_spmv<3>"
    assert bench.kernel_name("dg_vel", 2, pc, dg=True) == "k_dg_vcheb<2, double>"
    assert set(bench.SINGLE_KERNEL_FAMILIES) == {"spmv_K", "cheb_S_l0", "resid_S_l0", "schur_rhs", "schur_vel",
                                                 "dg_vel"}


def test_oracle_leg_reference_and_baseline_on_a_small_box():
    """The oracle leg on a 3D n = 6 log-normal box: its reference solution
    agrees with a direct solve, so a solution handed in as the direct solve
    gets per-field errors at the reference's accuracy and an oracle residual
    near zero; the CPU baseline names its sample and thread count."""
    import numpy as np

    import dpp_inputs as I
    from oracle import dpp as odpp
    prob = I.grf_problem(3, 6)
    S = odpp.assemble(prob)
    xd = odpp.solve_direct(S.K, S.f)
    base, errs = bench.oracle_leg(prob, gpu_iters=20, sample_iters=5,
                                  solutions={"direct": xd, "zero": np.zeros_like(xd)})
    assert base["kind"] == "oracle" and base["unit"] == "DOF/s" and base["value"] > 0
    assert base["cores"] >= 1 and "first 5 oracle FGMRES iterations" in base["sample"]
    assert all(errs["direct"][f] <= 1e-9 for f in ("u1", "p1", "u2", "p2"))
    assert errs["direct"]["oracle_residual"] <= 1e-12
    assert errs["zero"]["oracle_residual"] == 1.0
    base, _ = bench.oracle_leg(prob, gpu_iters=20, sample_iters=200, solutions={})
    assert "to 1e-8 from x = 0" in base["sample"]


def test_oracle_leg_on_a_dg_box():
    """The DG-VMS oracle leg (its own assembly and fieldsplit) on a 2D 6^2
    box: the reference agrees with a direct solve on every field."""
    import numpy as np

    import dpp_inputs as I
    from oracle import dg as odg
    from oracle import dpp as odpp
    prob = I.mms_problem(2, 6, elem="dg")
    S = odg.assemble(prob)
    xd = odpp.solve_direct(S.K, S.f)
    base, errs = bench.oracle_leg(prob, gpu_iters=30, sample_iters=4, solutions={"direct": xd})
    assert base["value"] > 0 and "block-Jacobi Chebyshev" in base["sample"]
    assert all(errs["direct"][f] <= 1e-9 for f in ("u1", "p1", "u2", "p2"))
    assert errs["direct"]["oracle_residual"] <= 1e-12


def test_oracle_batch_leg_stops_at_its_budget():
    import dpp_inputs as I
    probs = I.batch_configs(3, seed=7, nmin=4, nmax=8)
    base = bench.oracle_batch_leg(probs, budget_s=0.0)
    assert base["value"] > 0 and "the first 1 of the 3 instances" in base["sample"]
