"""The tuning table of workgroup shapes (dg_tuning_*): host logic, no GPU."""
import pytest

from paper_1208_4772_amd import dg
from paper_1208_4772_amd.dg import Tuning


@pytest.fixture(autouse=True)
def empty_table():
    Tuning.clear()
    yield
    Tuning.clear()


def test_set_lookup_and_clear():
    assert Tuning.lookup("gfx950", 4, "fp32", False) == 0
    Tuning.set("gfx950", 4, "fp32", False, 8)
    Tuning.set("gfx950", 4, "fp32", True, 2)
    Tuning.set("gfx950", 4, "bf16x3", False, 4)
    assert Tuning.lookup("gfx950", 4, "fp32", False) == 8
    assert Tuning.lookup("gfx950", 4, "fp32", True) == 2
    assert Tuning.lookup("gfx950", 4, "bf16x3", False) == 4
    # other architectures, orders and kinds are separate keys
    assert Tuning.lookup("gfx942", 4, "fp32", False) == 0
    assert Tuning.lookup("gfx950", 5, "fp32", False) == 0
    Tuning.clear()
    assert Tuning.lookup("gfx950", 4, "fp32", False) == 0


def test_save_and_load_round_trip(tmp_path):
    entries = {(p, prec, av): w for p, w in zip(range(1, 6), (2, 4, 8, 4, 2))
               for prec in ("fp32", "bf16x3") for av in (False, True)}
    for (p, prec, av), w in entries.items():
        Tuning.set("gfx950", p, prec, av, w)
    path = tmp_path / "tune.txt"
    assert Tuning.save(path) == len(entries)
    Tuning.clear()
    assert Tuning.load(path) == len(entries)
    for (p, prec, av), w in entries.items():
        assert Tuning.lookup("gfx950", p, prec, av) == w
    # the saved file loads again into the same table (merge, no duplicates)
    assert Tuning.load(path) == len(entries)
    path2 = tmp_path / "tune2.txt"
    assert Tuning.save(path2) == len(entries)
    assert path.read_text() == path2.read_text()


def test_load_merges_and_comments(tmp_path):
    Tuning.set("gfx950", 3, "fp32", False, 2)
    path = tmp_path / "t.txt"
    path.write_text("# comment\n\n  gfx950 3 2 0 8 10.5\ngfx950 5 3 1 4 0\n")
    assert Tuning.load(path) == 2
    assert Tuning.lookup("gfx950", 3, "fp32", False) == 8
    assert Tuning.lookup("gfx950", 5, "bf16x3", True) == 4


@pytest.mark.parametrize("line", ["gfx950 6 2 0 4 1.0",      # order out of range
                                  "gfx950 3 0 0 4 1.0",      # FP64 has no shape
                                  "gfx950 3 2 2 4 1.0",      # av not 0/1
                                  "gfx950 3 2 0 3 1.0",      # shape not 2/4/8
                                  "gfx950 3 2 0 4",          # missing field
                                  "gfx950 3 2 0 4 1.0 x"])   # trailing field
def test_malformed_file_is_rejected_whole(tmp_path, line):
    path = tmp_path / "bad.txt"
    path.write_text("gfx950 2 2 0 8 1.0\n" + line + "\n")
    with pytest.raises(dg.DGError) as e:
        Tuning.load(path)
    assert e.value.code == dg.DG_EINVAL and ":2:" in str(e.value)
    assert Tuning.lookup("gfx950", 2, "fp32", False) == 0


def test_bad_arguments():
    with pytest.raises(dg.DGError):
        Tuning.set("gfx950", 3, "fp64", False, 4)
    with pytest.raises(dg.DGError):
        Tuning.set("gfx950", 3, "fp32", False, 16)
    with pytest.raises(dg.DGError):
        Tuning.set("", 3, "fp32", False, 4)
    with pytest.raises(dg.DGError):
        Tuning.load("/nonexistent/dir/tune.txt")
