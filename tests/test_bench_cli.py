"""bench.py's command line on the CPU: more than one GPU is refused with a message before any
device work; the standard invocation (--gpus 1 --steps 20 --warmup 5) plans a run that fits the
full case's 1e6 primaries and the time limit, also checked before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

STANDARD_ARGS = ["--gpus", "1", "--steps", "20", "--warmup", "5"]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--no-cpu"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_standard_invocation_fits_the_job_and_the_time_limit():
    import bench
    from paper_2503_10263_amd import workloads as W
    pl = bench.plan(bench.parse(STANDARD_ARGS))
    assert (5 + 20) * pl["batch"] <= bench.N_FULL
    assert pl["batch"] == 40000                      # 1e6 // 25
    assert pl["slice_steps"] == W.FULL_SLICE_STEPS and pl["batched_queue"] == W.BATCHED_QUEUE
    assert pl["estimated_total_s"] <= bench.TIME_LIMIT_S - bench.MARGIN_S, pl["estimated_s"]


def test_standard_invocation_plan_without_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *STANDARD_ARGS, "--plan"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert '"batch": 40000' in r.stderr and r.stdout == ""


def test_oversized_runs_are_refused_before_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "20", "--warmup", "5",
                        "--batch", "131072", "--plan"], capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "exceed" in r.stderr


def test_defaults_are_small_and_within_the_job():
    import bench
    pl = bench.plan(bench.parse([]))
    assert (pl["warmup"] + pl["steps"]) * pl["batch"] <= bench.N_FULL
    assert (pl["slice_steps"] & (pl["slice_steps"] - 1)) == 0   # slices are a power of two


def test_profiled_constants_belong_to_these_kernel_sources():
    """The issue fraction, HBM bytes and batched issue fraction that bench.py reports were
    measured (rocprofv3, summaries under profiles/) on kernel sources of a stated hash; the bench
    reports them only while the sources still have that hash, and the committed profiles are
    those of the committed kernels."""
    import bench
    sha = bench.kernels_sha256()
    for name in ("VALU_ISSUE", "HBM_TRAFFIC", "BATCHED_VALU", "L2_COUNTERS"):
        assert getattr(bench, name)["kernels_sha256"] == sha, name
    for prof in ("transport_kernel_drain_full_case_sq.md", "transport_kernel_full_case_hbm.md",
                 "transport_kernel_full_case_ktrace.md", "transport_kernel_batched_fp32_batched_case.md",
                 "transport_kernel_l2_full_and_batched_case.md", "all_kernels_bench_steps20_warmup5_ktrace.md"):
        with open(os.path.join(ROOT, "profiles", prof)) as f:
            assert sha in f.read(), prof
