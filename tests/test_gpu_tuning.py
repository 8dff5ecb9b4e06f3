"""Tuner choices recorded on disk are what the tuners use once the file is read again (GPU).

mr_tuning_file points the library at a fresh file and makes the tuners drop the choices they keep
in memory, as a new process would start. A context (the FP64 sweep and defect tuners run on its
levels) and a mixed-precision solve (the FP32 sweep tuner) then leave their records in the file.
A planted record naming another candidate of the finest FP64 level is what the next context uses,
without timing: its schedule is the planted one.
"""
import pytest
import torch

from gpu_util import announce, require_gpu
from paper_1709_06350_amd import mr

pytestmark = pytest.mark.gpu

N = 64


def _code(kind, tm, tj, nch):
    """The record of a pipelined two-launch FP64 schedule on the N^3 level."""
    assert kind == mr.MR_SCHED_PIPELINED
    return [0, tm, tj, N // nch, N // tj, (N // 2) // tm, 1, 1, 0, 0, 0, 0, 0]


def test_recorded_choice_is_used_after_the_file_is_read_again(tmp_path):
    require_gpu()
    path = tmp_path / "tuning.txt"
    mr.tuning_file(str(path))
    try:
        announce("tuning: records")
        with mr.Context(N) as c:
            first = c.get_schedule(0)
            cands = c.schedule_candidates(0)
        d = torch.zeros((N, N, N), dtype=torch.float64, device="cuda")
        with mr.Context(N, precision=mr.PREC_MIXED) as m:
            m.solve(d, torch.zeros_like(d), check=False)
        lines = path.read_text().splitlines()
        kinds = {ln.split("|")[0] for ln in lines if not ln.startswith("#")}
        assert {"sweep64.v1", "lin32.v1"} <= kinds, kinds
        rec = [ln for ln in lines if ln.startswith("sweep64.v1|") and ln.split("|")[4] == str(N)]
        assert len(rec) == 1, lines
        # plant another pipelined candidate of the finest level and read the file again
        other = [tuple(x) for x in cands if x[0] == mr.MR_SCHED_PIPELINED and tuple(x) != tuple(first)]
        assert other, cands
        pick = other[len(other) // 2]
        key = "|".join(rec[0].split("|")[:5])
        planted = key + "|" + ",".join(str(v) for v in _code(*pick))
        path.write_text("\n".join(planted if ln == rec[0] else ln for ln in lines) + "\n")
        mr.tuning_file(str(path))
        announce(f"tuning: planted {pick}")
        with mr.Context(N) as c:
            assert c.get_schedule(0) == pick
        # a record that names no candidate is timed again (and replaced)
        path.write_text(key + "|0,3,5,7,1,1,1,1,0,0,0,0,0\n")
        mr.tuning_file(str(path))
        with mr.Context(N) as c:
            assert tuple(c.get_schedule(0)) in {tuple(x) for x in cands}
        assert "0,3,5,7" not in path.read_text()
    finally:
        mr.tuning_file(None)
