"""The measurement records: committed rocprofv3 summaries and the bench's use of them (CPU only).

The bench reports the smoother's HBM traffic from the committed counter summary only while that
summary was taken on the same kernel source and the same finest-level schedule; otherwise the
figure is null. The summaries themselves are short text files that give the commands which made
them, and those commands run committed files only.
"""
import importlib.util
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _profile_files():
    return sorted(os.listdir(PROFILES))


def test_profiles_are_short_text_summaries():
    files = _profile_files()
    assert files, "no profile summaries"
    for f in files:
        path = os.path.join(PROFILES, f)
        assert f.endswith((".txt", ".md")), f
        assert os.path.getsize(path) < 16 * 1024, f
        txt = open(path, encoding="utf-8").read()
        assert "rocprofv3" in txt, f"{f}: no command"


@pytest.mark.parametrize("name", _profile_files())
def test_profile_commands_run_committed_files(name):
    txt = open(os.path.join(PROFILES, name), encoding="utf-8").read()
    cmds = [ln for ln in txt.splitlines() if "&& rocprofv3 " in ln]
    assert cmds, name
    for ln in cmds:
        prog = ln.split(" -- ", 1)
        assert len(prog) == 2, ln
        # the profiled program comes directly after "--" and is the committed bench
        assert re.match(r"python3 <repo>/bench\.py(\s|$)", prog[1].strip()), ln
        assert "/tmp" in ln and "TMPDIR" in ln, ln


def test_traffic_needs_same_kernel_source_and_schedule(tmp_path):
    b = _bench()
    sched = "1,64,16,2"
    good = tmp_path / "pmc.txt"
    good.write_text(f"hbm_bytes_per_sweep: 4.4e+09\nschedule: {sched}\nkernel_source_hash: {b.kernel_hash()}\n")
    b.PROFILE_PMC = str(good)
    assert b.measured_traffic(sched) == pytest.approx(4.4e9)
    assert b.measured_traffic("1,64,8,2") is None
    stale = tmp_path / "stale.txt"
    stale.write_text(f"hbm_bytes_per_sweep: 4.4e+09\nschedule: {sched}\nkernel_source_hash: 0000000000000000\n")
    b.PROFILE_PMC = str(stale)
    assert b.measured_traffic(sched) is None
    b.PROFILE_PMC = str(tmp_path / "missing.txt")
    assert b.measured_traffic(sched) is None


def test_committed_sweep_counters_match_the_current_kernel():
    """The committed smoother counters were taken on the kernel source in the tree (else the bench's
    traffic figure would be null)."""
    b = _bench()
    txt = open(b.PROFILE_PMC, encoding="utf-8").read()
    m = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", txt)
    assert m and m.group(1) == b.kernel_hash()
    c = re.search(r"schedule:\s*([0-9,]+)", txt)
    assert c and b.measured_traffic(c.group(1)) > 0
