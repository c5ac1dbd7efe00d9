"""The device timeline (the library built with KP_TIMELINE) on a small
Allen-Cahn call: the stamps of every Arnoldi step come in the order of the
phase's work, and the phases add up to the call's event time.  Runs
`bench.py --timeline` in a child process, since the timeline build and the
default build cannot share one process's loader."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_timeline_of_a_small_call(tmp_path):
    print("timeline: bench.py --timeline, Allen-Cahn 256 x 256", flush=True)
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--timeline",
                          str(tmp_path), "--side", "256"], cwd=ROOT, capture_output=True,
                         text=True, timeout=180)
    assert res.returncode == 0, res.stderr[-3000:]
    for label in ("adaptive", "fixed_m64"):
        s = json.load(open(tmp_path / f"timeline_{label}.json"))
        assert s["info"]["status"] == 0
        # steps with a pending update: all but the first of each Arnoldi process
        n_upd = s["info"]["arnoldi_steps"] - s["info"]["substeps"]
        if label == "fixed_m64":
            assert s["arnoldi_steps"] == n_upd == 63
        else:
            assert 0.5 * n_upd <= s["arnoldi_steps"] <= n_upd
        m = s["step_mean_us"]
        assert 0 < m["release_seen_us"] < m["update_done_us"] <= m["halo_flags_us"]
        assert m["halo_flags_us"] < m["arrival_median_us"] <= m["arrival_last_us"]
        assert m["reduction_after_last_us"] > 0 and m["serial_us"] > 0
        total = s["steps_total_ms"] + sum(v["total_ms"] for v in s["other_phases"].values())
        # the phases cover the launch but for its start and end (init, last phase)
        assert 0.8 * s["event_ms"] <= total <= 1.01 * s["event_ms"]
