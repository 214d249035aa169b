"""The serving loop's admission policy (paper_2406_01821_amd/csrc/
serve_sched.h: the arena's first-fit allocator and the FIFO prefix a launch
takes) driven by a simulated executor on the host, no GPU: tests/sched/
sched_driver.cpp replays request streams from light load to constant
back-pressure and checks arena disjointness, arrival order, batch and
in-flight limits, back-pressure and completion after every step, and the
allocator's choices against a brute-force model.  Built with
AddressSanitizer and UndefinedBehaviorSanitizer."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_admission_policy_with_simulated_executor(tmp_path):
    exe = str(tmp_path / "sched_driver")
    src = os.path.join(ROOT, "tests", "sched", "sched_driver.cpp")
    inc = os.path.join(ROOT, "paper_2406_01821_amd", "csrc")
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-I", inc, src, "-o", exe, "-lm"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.strip().endswith("ok")
    print(r.stdout)
