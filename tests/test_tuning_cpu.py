"""CPU checks of the tuning table of the C library (ntt_tune_*): key grammar, value
ranges, all-or-nothing loading of a choices file, and that the committed choices
file for gfx950 (when present) is valid.  Pure host code: no GPU is touched."""
import os

import pytest

from paper_1407_3383_amd import ntt


@pytest.fixture()
def lib():
    if not os.path.exists(ntt.LIB_PATH):
        pytest.fail("libntt_mi355x.so not built")
    L = ntt.load()
    ntt.tune_clear()
    yield L
    ntt.tune_clear()
    if os.path.exists(ntt.TUNE_FILE):
        ntt.tune_load(ntt.TUNE_FILE)


@pytest.mark.parametrize("key,value", [
    ("split.w32.L24", 12), ("split.w32.L15", 14), ("split.w32.L26", 13), ("split.w64.L14", 12),
    ("split.w64.L21", 13), ("psplit.w32.L22", 12), ("psplit.w64.L20", 13),
    ("fused.single.max.w32", 14), ("fused.single.max.w32", 16), ("fused.single.max.w64", 13),
    ("single.split.w32.L13", 3), ("single.split.w32.L16", 3), ("single.split.w32.L11", 1), ("single.split.w32.L14", 0),
    ("single.split.w64.L15", 3), ("single.split.w64.L12", 2)])
def test_valid_choices_round_trip(lib, key, value):
    ntt.tune_set(key, value)
    assert ntt.tune_get(key) == value


@pytest.mark.parametrize("key,value", [
    ("split.w32.L24", 11), ("split.w32.L24", 15), ("split.w64.L20", 14), ("split.w32.L14", 12),
    ("split.w32.L27", 14), ("split.w16.L20", 12), ("split.w32.L20x", 12), ("fused.single.max.w32", 17),
    ("fused.single.max.w64", 16), ("fused.max.w32", 15), ("", 1), ("row.w32.L20", 12),
    ("single.split.w32.L16", 2), ("single.split.w32.L12", 3), ("single.split.w32.L17", 3), ("single.split.w32.L10", 0),
    ("single.split.w64.L15", 2), ("single.split.w32.L14", 4)])
def test_invalid_choices_are_refused(lib, key, value):
    with pytest.raises(ntt.NTTError):
        ntt.tune_set(key, value)
    assert ntt.tune_get(key) is None


def test_unset_key_reads_as_none_and_clear_forgets(lib):
    assert ntt.tune_get("split.w32.L20") is None
    ntt.tune_set("split.w32.L20", 13)
    ntt.tune_clear()
    assert ntt.tune_get("split.w32.L20") is None


def test_load_applies_every_line(lib, tmp_path):
    f = tmp_path / "choices.txt"
    f.write_text("# header\n\nsplit.w32.L20 12   # ms: ...\n  psplit.w64.L18 13\nfused.single.max.w32 15\n")
    ntt.tune_load(str(f))
    assert ntt.tune_get("split.w32.L20") == 12
    assert ntt.tune_get("psplit.w64.L18") == 13
    assert ntt.tune_get("fused.single.max.w32") == 15


@pytest.mark.parametrize("bad", ["split.w32.L20 12\nsplit.w32.L21 99\n", "split.w32.L20\n",
                                 "split.w32.L20 12 13\n", "nonsense 1\n"])
def test_load_is_all_or_nothing(lib, tmp_path, bad):
    f = tmp_path / "bad.txt"
    f.write_text(bad)
    with pytest.raises(ntt.NTTError):
        ntt.tune_load(str(f))
    assert ntt.tune_get("split.w32.L20") is None


def test_load_missing_file(lib, tmp_path):
    with pytest.raises(ntt.NTTError):
        ntt.tune_load(str(tmp_path / "absent.txt"))


def test_committed_choices_file_is_valid(lib):
    if not os.path.exists(ntt.TUNE_FILE):
        pytest.skip("no tuned choices committed for gfx950")
    ntt.tune_load(ntt.TUNE_FILE)
    keys = [ln.split()[0] for ln in open(ntt.TUNE_FILE) if ln.split() and not ln.lstrip().startswith("#")]
    assert keys and all(ntt.tune_get(k) is not None for k in keys)
