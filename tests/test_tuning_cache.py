"""The persistent record of tuner choices (host code only; no GPU).

The library's tuners look a recorded choice up by (kind, architecture, device, compute units, n)
and record new ones; these tests drive the same store through mr_tuning_store / mr_tuning_lookup
and check the round trip through the file, the key's parts, the file's format and that unreadable
lines are skipped.
"""
import os

import pytest

from paper_1709_06350_amd import mr

ARCH = "gfx950:sramecc+:xnack-"
DEV = "AMD Instinct MI355X"


@pytest.fixture
def tfile(tmp_path):
    path = tmp_path / "sub" / "tuning.txt"
    mr.tuning_file(str(path))
    yield path
    mr.tuning_file(None)


def test_round_trip_through_the_file(tfile):
    vals = [1, 64, 16, 32, 32, 4, 1, 1, 0, 0, 0, 0, 0]
    mr.tuning_store("sweep64.v1", ARCH, DEV, 256, 512, vals)
    assert tfile.exists(), "the record is written at once (parent folders created)"
    assert mr.tuning_lookup("sweep64.v1", ARCH, DEV, 256, 512) == vals
    # forget the in-memory records and read the file again (a later process)
    mr.tuning_file(str(tfile))
    assert mr.tuning_lookup("sweep64.v1", ARCH, DEV, 256, 512) == vals
    text = tfile.read_text()
    assert f"sweep64.v1|{ARCH}|{DEV}|256|512|" + ",".join(map(str, vals)) in text
    assert text.startswith("#")


def test_every_part_of_the_key_counts(tfile):
    mr.tuning_store("lin32.v1", ARCH, DEV, 256, 256, [7, 8, 9])
    assert mr.tuning_lookup("lin32.v1", ARCH, DEV, 256, 256) == [7, 8, 9]
    assert mr.tuning_lookup("lin32.v1", ARCH, DEV, 256, 512) is None          # n
    assert mr.tuning_lookup("lin32.v1", ARCH, DEV, 304, 256) is None          # compute units
    assert mr.tuning_lookup("lin32.v1", "gfx942", DEV, 256, 256) is None       # architecture
    assert mr.tuning_lookup("lin32.v1", ARCH, "MI300X", 256, 256) is None      # device
    assert mr.tuning_lookup("lin32.v2", ARCH, DEV, 256, 256) is None           # kind / format version
    # a later record under the same key replaces the earlier one
    mr.tuning_store("lin32.v1", ARCH, DEV, 256, 256, [1, -2])
    mr.tuning_file(str(tfile))
    assert mr.tuning_lookup("lin32.v1", ARCH, DEV, 256, 256) == [1, -2]


def test_unreadable_lines_are_skipped(tfile):
    tfile.parent.mkdir(parents=True, exist_ok=True)
    tfile.write_text("# comment\n"
                     "garbage without separators\n"
                     f"adj64.v1|{ARCH}|{DEV}|256|128|1,x,3\n"
                     f"adj64.v1|{ARCH}|{DEV}|256|64|\n"
                     f"adj64.v1|{ARCH}|{DEV}|256|256|64,8,32,1\n")
    mr.tuning_file(str(tfile))
    assert mr.tuning_lookup("adj64.v1", ARCH, DEV, 256, 256) == [64, 8, 32, 1]
    assert mr.tuning_lookup("adj64.v1", ARCH, DEV, 256, 128) is None
    assert mr.tuning_lookup("adj64.v1", ARCH, DEV, 256, 64) is None


def test_separators_in_names_do_not_break_records(tfile):
    mr.tuning_store("blin32.v1", ARCH, "odd|name", 8, 16, [3])
    mr.tuning_file(str(tfile))
    assert mr.tuning_lookup("blin32.v1", ARCH, "odd|name", 8, 16) == [3]


def test_no_file_keeps_records_in_memory_only(tmp_path):
    mr.tuning_file("")
    try:
        assert mr.tuning_file_path() == ""
        mr.tuning_store("defect64.v1", ARCH, DEV, 256, 32, [16, 8, 2])
        assert mr.tuning_lookup("defect64.v1", ARCH, DEV, 256, 32) == [16, 8, 2]
        assert not any(tmp_path.iterdir())
    finally:
        mr.tuning_file(None)


def test_default_location_follows_the_environment(tmp_path, monkeypatch):
    path = tmp_path / "env_tuning.txt"
    monkeypatch.setenv("MR_TUNING_FILE", str(path))
    mr.tuning_file(None)
    try:
        assert mr.tuning_file_path() == str(path)
        monkeypatch.delenv("MR_TUNING_FILE")
        monkeypatch.setenv("XDG_CACHE_HOME", str(tmp_path / "xdg"))
        mr.tuning_file(None)
        assert mr.tuning_file_path() == os.path.join(str(tmp_path / "xdg"), "paper_1709_06350_amd", "tuning.txt")
    finally:
        mr.tuning_file(None)


def test_bad_arguments_are_errors(tfile):
    with pytest.raises(mr.MRError):
        mr.tuning_store("k", ARCH, DEV, 256, 0, [1])
    with pytest.raises(mr.MRError):
        mr.tuning_store("k", ARCH, DEV, 256, 8, [])
    mr.tuning_store("k", ARCH, DEV, 256, 8, [1, 2, 3])
    with pytest.raises(mr.MRError):
        mr.tuning_lookup("k", ARCH, DEV, 256, 8, max_count=2)


def test_shipped_defaults_are_consulted_after_the_record_file(tmp_path, monkeypatch):
    """A key missing from the record file is taken from the shipped choices ($MR_TUNING_DEFAULTS
    here, tuning_defaults.txt beside the library otherwise); a record in the file wins; the shipped
    file is never written."""
    shipped = tmp_path / "defaults.txt"
    shipped.write_text(f"# shipped\nsweep64.v1|{ARCH}|288GiB|256|512|0,64,16,256,32,4,1,1,0,0,0,0,0\n")
    before = shipped.read_text()
    monkeypatch.setenv("MR_TUNING_DEFAULTS", str(shipped))
    user = tmp_path / "user.txt"
    mr.tuning_file(str(user))
    try:
        assert mr.tuning_lookup("sweep64.v1", ARCH, "288GiB", 256, 512) == [0, 64, 16, 256, 32, 4, 1, 1, 0, 0, 0, 0, 0]
        mr.tuning_store("sweep64.v1", ARCH, "288GiB", 256, 512, [1, 2, 3])
        assert mr.tuning_lookup("sweep64.v1", ARCH, "288GiB", 256, 512) == [1, 2, 3]
        assert shipped.read_text() == before
        assert "sweep64.v1" in user.read_text()
        monkeypatch.setenv("MR_TUNING_DEFAULTS", "")
        mr.tuning_file(str(tmp_path / "other.txt"))
        assert mr.tuning_lookup("sweep64.v1", ARCH, "288GiB", 256, 512) is None
    finally:
        monkeypatch.delenv("MR_TUNING_DEFAULTS", raising=False)
        mr.tuning_file(None)


def test_shipped_defaults_file_parses_and_names_this_device_kind():
    """The committed defaults are records of the library's tuner kinds for gfx950 devices."""
    path = os.path.join(os.path.dirname(mr.__file__), "tuning_defaults.txt")
    if not os.path.exists(path):
        pytest.skip("no shipped defaults")
    kinds = set()
    for ln in open(path):
        if ln.startswith("#") or not ln.strip():
            continue
        parts = ln.strip().split("|")
        assert len(parts) == 6, ln
        kinds.add(parts[0])
        assert parts[1].startswith("gfx950")
        assert all(v.lstrip("-").isdigit() for v in parts[5].split(","))
    assert {"sweep64.v1", "lin32.v1"} <= kinds
