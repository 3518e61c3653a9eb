"""Host-side parts of bench.py (CPU only): the refusal of more than one GPU,
and the CPU-baseline record, which times the oracle on a bounded sample."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_cpu_baseline_record():
    """A short sample: the FFT-PCGS oracle at n = 2^10 on the first levels,
    the dense-LU sweep beside it (median of repeats, every host core); the
    fields the bench line carries."""
    sys.path.insert(0, ROOT)
    import bench
    rec = bench.cpu_baseline(1 << 10, 16, 1e-10, budget_s=1.0, lu_sizes=(64, 128), lu_reps=3)
    assert rec["kind"] == "oracle" and rec["unit"] == "level-solves/s" and rec["cores"] == 1
    assert rec["host_cores"] == bench.host_cores() >= 1
    assert rec["value"] > 0 and "FFT-PCGS oracle" in rec["sample"]
    lu = rec["dense_lu"]
    assert lu["cores"] == rec["host_cores"] and [r["n"] for r in lu["sweep"]] == [64, 128]
    for r in lu["sweep"]:
        assert r["repeats"] == 3 and r["seconds_per_level"] > 0
        assert abs(r["level_solves_per_s"] * r["seconds_per_level"] - 1) < 1e-12
    big = lu["sweep"][-1]
    assert abs(lu["value_extrapolated"] - big["level_solves_per_s"] * (128 / 1024) ** 3) <= 1e-9 * lu["value_extrapolated"]


def test_acceptance_summary():
    """The acceptance record of a march: failed levels by status code, the
    largest backward error and true residual among the levels that computed
    them (-1 = not computed), total restarts."""
    sys.path.insert(0, ROOT)
    import bench
    st = [{"code": 0, "backward_err": 3e-14, "relres_true": 2e-9, "restarts": 0},
          {"code": -9, "backward_err": 5e-12, "relres_true": 4e-7, "restarts": 3},
          {"code": 0, "backward_err": -1.0, "relres_true": -1.0, "restarts": 1}]
    a = bench.acceptance(st)
    assert a == {"levels": 3, "failed_levels": 1, "max_backward_err": 5e-12, "max_relres_true": 4e-7,
                 "restarts": 4}
    assert bench.acceptance(st[2:])["max_backward_err"] is None


def test_path_bytes_model():
    """One level: k CGS iterations at 416n bytes each plus the right-hand side
    at 112n; two levels add the first block's history sweep (u^0 read, the
    block's sums written)."""
    sys.path.insert(0, ROOT)
    import bench
    n = 1000
    assert bench.path_bytes(n, 16, 1, [7]) == 416 * n * 7 + 112 * n
    assert bench.path_bytes(n, 16, 2, [7, 5]) == 416 * n * 12 + 112 * n * 2 + 8 * n * (1 + 8)


def test_fused_bytes_model():
    """The fused path: 45 units of 8n per CGS iteration, 20 per level, plus
    the history (here none: one level)."""
    sys.path.insert(0, ROOT)
    import bench
    n = 1000
    assert bench.fused_bytes(n, 16, 1, [7]) == 8 * n * (45 * 7 + 20)


def test_iteration_summary_and_network_cost():
    """Iteration distribution of a march, and the network's cost in CGS
    iterations from the line through the previous-level and extrapolated
    points (level time = c + t_it * iterations)."""
    sys.path.insert(0, ROOT)
    import bench
    s = bench.iteration_summary([4, 6, 5, 9, 6])
    assert s["mean"] == 6.0 and s["p50"] == 6.0 and s["max"] == 9.0
    assert abs(s["p90"] - 7.8) < 1e-12  # linear interpolation between 6 and 9
    c, t_it = 0.2e-3, 0.05e-3
    prev, extrap = (c + 10 * t_it, 10.0), (c + 7 * t_it, 7.0)
    # a network guess worth 6 iterations whose inference costs 0.75 of one
    net = (c + 6 * t_it + 0.75 * t_it, 6.0)
    assert abs(bench.net_cost_iterations(prev, extrap, net) - 0.75) < 1e-9
    assert bench.net_cost_iterations(prev, (c + 10 * t_it, 10.0), net) is None
