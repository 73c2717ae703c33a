"""Tuning database on the CPU: load, lookup through the planner, save, clear."""
import pytest

from paper_2207_06803_amd import fftc


@pytest.fixture(autouse=True)
def clean_db():
    fftc.tune_clear()
    yield
    fftc.tune_clear()


def test_loaded_entry_drives_the_planner(tmp_path):
    default, _ = fftc.factorize(1024)
    db = tmp_path / "tune.txt"
    key = fftc.tune_key()
    arch, toolchain = key.split()
    assert arch == "gfx950" and toolchain.startswith("hip")
    db.write_text(f"{key} c64 1024 16,4,16 0.010\n"
                  f"{key} c64 512 3,3,3 0.1\n"            # does not multiply to 512: ignored
                  f"gfx942 {toolchain} c64 2048 16,16,8 0.1\n"  # other architecture: ignored
                  f"{arch} hip0.0.0 c64 2048 16,16,8 0.1\n"     # other toolchain: ignored
                  "gfx950 c64 2048 16,16,8 0.1\n"        # old format without the toolchain: ignored
                  f"{key} c64 256 6,6 0.1\n"              # radix 6 unsupported: ignored
                  f"{key} c64 64 4,16 0.1 extra\n"        # trailing field: ignored
                  f"{key} c128 64 4,16 0.001\n")
    assert fftc.tune_load(str(db)) == 2
    assert fftc.factorize(1024)[0] == [16, 4, 16]
    assert fftc.factorize(64, "c128")[0] == [4, 16]
    assert fftc.factorize(512)[0] == fftc.factorize(512)[0]
    out = tmp_path / "saved.txt"
    assert fftc.tune_save(str(out)) == 2
    lines = sorted(out.read_text().split("\n"))
    assert any(l.startswith(f"{key} c64 1024 16,4,16 ") for l in lines)
    fftc.tune_clear()
    assert fftc.factorize(1024)[0] == default
    assert fftc.tune_load(str(out)) == 2
    assert fftc.factorize(1024)[0] == [16, 4, 16]


def test_missing_file_is_an_error(tmp_path):
    with pytest.raises(fftc.FFTCError) as e:
        fftc.tune_load(str(tmp_path / "nope.txt"))
    assert e.value.status == 1


def test_autotune_argument_checks_on_host():
    with pytest.raises(fftc.FFTCError) as e:
        fftc.autotune(11, 4)
    assert e.value.status == 2
    with pytest.raises(fftc.FFTCError) as e:
        fftc.autotune(1 << 16, 4)      # two-pass length: not a single-kernel candidate
    assert e.value.status == 2
    with pytest.raises(fftc.FFTCError) as e:
        fftc.autotune(3 << 13, 4)      # past the single-kernel limit, no compiled wide list
    assert e.value.status == 2
    with pytest.raises(fftc.FFTCError) as e:
        fftc.autotune(64, 0)
    assert e.value.status == 1


def test_mixed_launch_mode_argument_checks_on_host():
    assert fftc.lib.fftc_plan_mixed_set_launch(None, fftc.MIXED_LAUNCH_DIRECT) == 1  # NULL plan


def test_mixed_plan_argument_checks_on_host():
    for bad in ([8, 11], [8, 8192], [0], []):
        with pytest.raises(fftc.FFTCError) as e:
            fftc.plan_mixed(bad)
        assert e.value.status in (1, 2), bad
