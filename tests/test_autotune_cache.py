"""The autotuner's persistent cache on the host (no GPU needed): an empty
dataset has a key without reading device memory, so the lookup path --
missing file, valid file, corrupt files -- runs here through the C ABI."""
import json
import os

import pytest
import torch

from paper_2312_02756_amd import glv

DEFAULT_FWD = (256, 32, 128, 512)
DEFAULT_BWD = (128, 64, 128, 512)


@pytest.fixture
def cache(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("GLV_AUTOTUNE_CACHE", str(path))
    glv.glv_autotune_forget()
    yield path
    glv.glv_autotune_forget()


def _write(path, entries, fmt="glv-autotune-1"):
    path.write_text(json.dumps({"format": fmt, "entries": [{"key": k, "tiling": list(t)} for k, t in entries]}))


def test_key_of_an_empty_dataset_names_its_parts():
    key = glv.glv_autotune_key(None, torch.float32, "PtEtaPhiM", "compensated")
    arch, dt, co, what, sig = key.split("|")
    assert (dt, co, what, sig) == ("f32", "PtEtaPhiM", "fwd-compensated", "e-1")
    assert glv.glv_autotune_key(None, backward=True).split("|")[3] == "bwd"


def test_missing_file_falls_back_to_the_default(cache, capfd):
    t, found = glv.glv_autotune_lookup(None)
    assert (t, found) == (DEFAULT_FWD, False)
    assert "does not exist" in capfd.readouterr().err
    assert not cache.exists()
    t, found = glv.glv_autotune_lookup(None, backward=True)
    assert (t, found) == (DEFAULT_BWD, False)


def test_valid_file_is_used_and_becomes_the_current_choice(cache):
    kf = glv.glv_autotune_key(None)
    kb = glv.glv_autotune_key(None, backward=True)
    _write(cache, [(kf, (64, 16, 64, 128)), (kb, (64, 64, 256, 1024))])
    assert glv.glv_autotune_lookup(None) == ((64, 16, 64, 128), True)
    assert glv.glv_current_tiling(torch.float64, "PtEtaPhiM", "plain") == (64, 16, 64, 128)
    assert glv.glv_autotune_lookup(None, backward=True) == ((64, 64, 256, 1024), True)
    assert glv.glv_current_tiling_bwd(torch.float64, "PtEtaPhiM") == (64, 64, 256, 1024)
    # another dtype has another key: not found, the default
    assert glv.glv_autotune_lookup(None, dtype=torch.float32) == (DEFAULT_FWD, False)
    # the process keeps the choice after the file goes away, until it forgets
    cache.unlink()
    assert glv.glv_autotune_lookup(None) == ((64, 16, 64, 128), True)
    glv.glv_autotune_forget()
    assert glv.glv_autotune_lookup(None) == (DEFAULT_FWD, False)
    assert glv.glv_current_tiling(torch.float64, "PtEtaPhiM", "plain") == DEFAULT_FWD


@pytest.mark.parametrize("bad", ["truncated", "format", "duplicate", "tiling", "lds", "trailing", "type", "empty"])
def test_corrupt_file_is_reported_ignored_and_kept(cache, capfd, bad):
    key = glv.glv_autotune_key(None)
    good = json.dumps({"format": "glv-autotune-1", "entries": [{"key": key, "tiling": [64, 16, 64, 128]}]})
    text = {
        "truncated": good[:-5],
        "format": good.replace("glv-autotune-1", "glv-autotune-0"),
        "duplicate": json.dumps({"format": "glv-autotune-1", "entries": [{"key": key, "tiling": [64, 16, 64, 128]},
                                                                         {"key": key, "tiling": [64, 16, 64, 128]}]}),
        "tiling": good.replace("[64, 16, 64, 128]", "[100, 16, 64, 128]"),
        "lds": good.replace("[64, 16, 64, 128]", "[512, 64, 4096, 4096]"),
        "trailing": good + " x",
        "type": good.replace("[64, 16, 64, 128]", '[64, "16", 64, 128]'),
        "empty": "",
    }[bad]
    cache.write_text(text)
    t, found = glv.glv_autotune_lookup(None)
    assert (t, found) == (DEFAULT_FWD, False)
    assert "corrupt" in capfd.readouterr().err
    assert cache.read_text() == text  # never rewritten


def test_empty_entries_and_whitespace_are_valid(cache, capfd):
    cache.write_text('\n{ "format" : "glv-autotune-1" ,\n "entries" : [ ] }\n')
    assert glv.glv_autotune_lookup(None) == (DEFAULT_FWD, False)
    err = capfd.readouterr().err
    assert "corrupt" not in err and "has no tiling" in err


def test_no_cache_variable(monkeypatch, capfd):
    monkeypatch.delenv("GLV_AUTOTUNE_CACHE", raising=False)
    glv.glv_autotune_forget()
    assert glv.glv_autotune_lookup(None) == (DEFAULT_FWD, False)
    assert "GLV_AUTOTUNE_CACHE not set" in capfd.readouterr().err
