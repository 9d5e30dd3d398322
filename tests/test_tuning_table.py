"""The autotuner's tuning table across processes (host only, no GPU):
keys by architecture, refinement flag and batch class (floor log2 of total
pairs and of problem count, depth bucket <= 9 / <= 16 / deeper), file round
trip, and rejection of malformed files without a partial merge."""
import pytest

from paper_1811_03374_amd import binding

HEADER = "fiberhit-tuning 1\n"


@pytest.fixture(autouse=True)
def empty_table():
    binding.clear_tuning()
    yield
    binding.clear_tuning()


def write(tmp_path, text, name="t.txt"):
    p = tmp_path / name
    p.write_text(text)
    return str(p)


def test_entries_are_found_by_class(tmp_path):
    # gfx950, plain, 2^20..2^21-1 pairs, 256..511 scenes, depth bucket 2 (> 16)
    binding.load_tuning(write(tmp_path, HEADER + "gfx950 0 20 8 2 56 0 1\n"
                                                 "gfx950 1 20 8 2 8 4 0\n"
                                                 "gfx950 0 20 8 0 32 5 0\n"))
    want = {"refill": 56, "waves_per_simd": 0, "stack": 1}
    assert binding.lookup_tuning("gfx950", 1 << 20, 256, 22) == want
    assert binding.lookup_tuning("gfx950", (1 << 21) - 1, 511, 17) == want
    assert binding.lookup_tuning("gfx950", 1 << 21, 256, 22) is None          # next pair class
    assert binding.lookup_tuning("gfx950", 1 << 20, 512, 22) is None          # next scene class
    assert binding.lookup_tuning("gfx950", 1 << 20, 256, 16) is None          # bucket 1
    assert binding.lookup_tuning("gfx950", 1 << 20, 256, 9) == {"refill": 32, "waves_per_simd": 5, "stack": 0}
    assert binding.lookup_tuning("gfx950", 1 << 20, 256, 10) is None
    assert binding.lookup_tuning("gfx950", 1 << 20, 256, 22, refine=True) == {"refill": 8, "waves_per_simd": 4,
                                                                                 "stack": 0}
    assert binding.lookup_tuning("gfx942", 1 << 20, 256, 22) is None          # another architecture


def test_round_trip_and_merge(tmp_path):
    a = write(tmp_path, HEADER + "gfx950 0 13 0 2 48 5 0\ngfx950 0 23 8 1 56 0 1\n", "a.txt")
    binding.load_tuning(a)
    out = str(tmp_path / "out.txt")
    binding.save_tuning(out)
    lines = open(out).read().splitlines()
    assert lines[0] == HEADER.strip()
    assert sorted(lines[1:]) == ["gfx950 0 13 0 2 48 5 0", "gfx950 0 23 8 1 56 0 1"]
    binding.clear_tuning()
    assert binding.lookup_tuning("gfx950", 1 << 13, 1, 22) is None
    binding.load_tuning(out)
    assert binding.lookup_tuning("gfx950", 1 << 13, 1, 22) == {"refill": 48, "waves_per_simd": 5, "stack": 0}
    # a later file replaces entries of the same key and keeps the others
    binding.load_tuning(write(tmp_path, HEADER + "gfx950 0 13 0 2 32 4 1\n", "b.txt"))
    assert binding.lookup_tuning("gfx950", 1 << 13, 1, 22) == {"refill": 32, "waves_per_simd": 4, "stack": 1}
    assert binding.lookup_tuning("gfx950", 1 << 23, 256, 12) == {"refill": 56, "waves_per_simd": 0, "stack": 1}


@pytest.mark.parametrize("text", [
    "",                                             # no header
    "fiberhit-tuning 2\n",                          # unknown version
    HEADER + "gfx950 0 20 8 2 56 0\n",              # missing field
    HEADER + "gfx950 0 20 8 2 56 0 1 7\n",          # extra field
    HEADER + "gfx950 0 20 8 2 65 0 0\n",            # refill out of range
    HEADER + "gfx950 0 20 8 2 56 17 0\n",           # waves per SIMD out of range
    HEADER + "gfx950 0 20 8 2 56 0 2\n",            # unknown stack layout
    HEADER + "gfx950 0 20 8 3 56 0 0\n",            # unknown depth bucket
    HEADER + "gfx950 2 20 8 2 56 0 0\n",            # refine flag not 0/1
])
def test_malformed_files_merge_nothing(tmp_path, text):
    good = HEADER + "gfx950 0 20 8 2 56 0 1\n"
    with pytest.raises(binding.FiberHitError):
        binding.load_tuning(write(tmp_path, good + text[len(HEADER):] if text.startswith(HEADER) else text))
    assert binding.lookup_tuning("gfx950", 1 << 20, 256, 22) is None


def test_missing_file_and_bad_arguments(tmp_path):
    with pytest.raises(binding.FiberHitError):
        binding.load_tuning(str(tmp_path / "absent.txt"))
    with pytest.raises(binding.FiberHitError):
        binding.save_tuning(str(tmp_path / "no_such_dir" / "t.txt"))
    assert binding.lookup_tuning("gfx950", -1, 1, 9) is None
    assert binding.lookup_tuning("gfx950", 1, 0, 9) is None
    assert binding.lookup_tuning("gfx950", 1, 1, 24) is None
