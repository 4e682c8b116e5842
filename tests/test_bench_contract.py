"""bench.py's contract on a host without a GPU: more than one GPU is refused with a message and
exit status 2 for every workload, before anything touches a device."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("workload", ["grf128", "pts256", "pts512", "train"])
def test_more_than_one_gpu_is_refused(workload):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--workload", workload,
                        "--no-cpu"], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2, (r.returncode, r.stderr[-500:])
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_counter_summaries_follow_the_code_not_its_comments():
    """The committed counter summaries stay valid across comment edits of the HIP sources and are
    dropped once the code changes: the hash covers the code with comments left out."""
    sys.path.insert(0, ROOT)
    import bench
    src = 'int a = 1; // one\n/* block\n comment */ const char *s = "a//b /* c */"; char c = \'/\';\n\n  f(a);\n'
    same = 'int a = 1;\n// another comment\nconst char *s = "a//b /* c */"; char c = \'/\';\n  f(a);  /* x */\n'
    other = src.replace("f(a)", "g(a)")
    assert bench._code_only(src) == bench._code_only(same)
    assert '"a//b /* c */"' in bench._code_only(src)
    assert bench._code_only(other) != bench._code_only(src)
    # the committed summaries belong to the code as it stands
    for wl in ("pts512", "grf128"):
        assert bench.measured_counters("step_queue_kernel<double>", wl) is not None, wl
