"""Tile tuner cache handling on the host: a missing, corrupt or partial cache
falls back to the deterministic defaults (no GPU needed)."""
import json

from paper_2602_03438_amd import autotune


def test_corrupt_cache_gives_defaults(tmp_path, monkeypatch):
    p = tmp_path / "tune_cache.json"
    p.write_text('{"gfx950/b=512/f64g/zgemm": {"best": 4, ')          # truncated JSON
    monkeypatch.setenv("NEGF_TUNE_CACHE", str(p))
    assert autotune.lookup(512, 3) == autotune.DEFAULT


def test_missing_cache_gives_defaults(tmp_path, monkeypatch):
    monkeypatch.setenv("NEGF_TUNE_CACHE", str(tmp_path / "absent.json"))
    assert autotune.lookup(256) == autotune.DEFAULT


def test_partial_cache_takes_what_it_has(tmp_path, monkeypatch):
    p = tmp_path / "tune_cache.json"
    p.write_text(json.dumps({autotune.key(384, "f64", "zinv"): {"best": 32}}))
    monkeypatch.setenv("NEGF_TUNE_CACHE", str(p))
    got = autotune.lookup(384)
    assert got["inv_nb"] == 32
    assert got["gemm_tile"] == autotune.DEFAULT["gemm_tile"]
    assert got["gemm_tile_f32"] == autotune.DEFAULT["gemm_tile_f32"]


def test_shipped_cache_is_valid():
    c = autotune.load_cache()
    assert c, "the shipped tune_cache.json is empty or unreadable"
    for k, v in c.items():
        assert k.startswith(autotune.ARCH + "/b="), k
        if k.endswith("/step"):
            assert v["best"]["gemm_tile"] in (1, 2, 3, 4, 5, 6) and v["best"]["inv_nb"] in (16, 32), (k, v)
        else:
            assert int(v["best"]) in (1, 2, 3, 4, 5, 6, 16, 32), (k, v)


def test_step_entry_overrides_kernel_timings(tmp_path, monkeypatch):
    """A whole-step timing decides over the kernel timings in isolation (for the
    complex-product form it was timed with)."""
    p = tmp_path / "tune_cache.json"
    p.write_text(json.dumps({autotune.key(640, "f64g", "zgemm"): {"best": 4},
                             autotune.key(640, "f64", "zinv"): {"best": 16},
                             autotune.key(640, "f64g", "step"): {"best": {"gemm_tile": 1, "inv_nb": 32}}}))
    monkeypatch.setenv("NEGF_TUNE_CACHE", str(p))
    got = autotune.lookup(640, 3)
    assert got["gemm_tile"] == 1 and got["inv_nb"] == 32
    got4 = autotune.lookup(640, 4)            # no step (nor product) entry for the four-product form
    assert got4["gemm_tile"] == autotune.DEFAULT["gemm_tile"] and got4["inv_nb"] == 16
