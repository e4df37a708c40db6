"""CPU checks of bench.py's contract that need no GPU: the refusal of more than
one GPU, the HBM traffic it reads from the committed counter summary, and the
oracle baseline sampler on a small workload."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and r.stdout == ""
    assert "one GPU" in r.stderr


def test_recorded_traffic_matches_the_algorithmic_bytes():
    """The counter summary of coupling64 at 1,310,720 triangles: either it was
    taken on the current kernel source (then its bytes are within 5% above the
    algorithmic 1,710,034 blocks x 64 x 64 x 4 bytes) or the bench reports none."""
    t = bench.recorded_traffic("sphere1310k_m4_f32")
    algorithmic = 1710034 * 64 * 64 * 4.0
    assert t is None or 1.0 <= t / algorithmic <= 1.05
    assert bench.recorded_traffic("no_such_workload") is None


def test_cpu_baseline_child_on_a_small_mesh():
    """The oracle baseline runs in a child interpreter on one core and on two
    (each core timing its own sample; their rates add)."""
    class A:
        workload = "sphere5120_m4_f64"
    for cores in (1, 2):
        out = bench.cpu_baseline(A, "sphere5120_m4_f64", 300000, 60000, cores, 1.0)
        assert out["kind"] == "oracle" and out["cores"] == cores and out["unit"] == "H2 matvecs/s", out
        est = out["est_seconds_per_matvec_per_core"]
        assert len(est) == cores and out["value"] > 0
        assert abs(out["value"] - sum(1.0 / e for e in est)) < 1e-9 * out["value"]
        assert "subtree" in out["sample"]


def test_profile_commands_run_committed_files_with_known_flags():
    """Every rocprofv3 command quoted in profiles/ runs bench.py from the
    repository with options bench.py still accepts."""
    import re
    import subprocess
    helptext = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True,
                              text=True, timeout=120).stdout
    prof = os.path.join(ROOT, "profiles")
    names = sorted(os.listdir(prof))
    assert names
    for name in names:
        text = open(os.path.join(prof, name)).read()
        cmds = [ln for ln in text.splitlines() if ln.strip().startswith("timeout") and "rocprofv3" in ln]
        assert cmds, name
        for c in cmds:
            prog = c.split(" -- ", 1)[1].split()
            assert prog[0] == "python3" and prog[1] == "$R/bench.py", (name, c)
            for flag in re.findall(r"(--[a-z][a-z0-9-]*)", " ".join(prog[2:])):
                assert flag in helptext, (name, flag)
