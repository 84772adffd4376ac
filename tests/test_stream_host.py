"""The stream's resume point on the host (no GPU): the progress file round trip,
refusal of another stream's file, atomic replacement, and the chunk files."""
import json
import os

import numpy as np
import pytest

from paper_2208_14567_amd.stream import NpzSink, Progress, StreamConfig


def test_progress_round_trip(tmp_path):
    cfg = StreamConfig(seed=5, chunks=25)
    p = Progress(str(tmp_path / "progress.json"))
    assert p.load(cfg) is None
    p.save(cfg, 3, {"candidates": 12, "valid": 4})
    st = p.load(cfg)
    assert st["next_chunk"] == 3 and st["totals"] == {"candidates": 12, "valid": 4}
    assert not os.path.exists(p.path + ".tmp")
    p.save(cfg, 4, {"candidates": 16, "valid": 5})
    assert p.load(cfg)["next_chunk"] == 4


def test_progress_refuses_another_stream(tmp_path):
    p = Progress(str(tmp_path / "progress.json"))
    p.save(StreamConfig(seed=5, chunks=25), 3, {})
    for other in (StreamConfig(seed=6, chunks=25), StreamConfig(seed=5, chunks=25, chunk=1000),
                  StreamConfig(seed=5, chunks=25, rules=True)):
        with pytest.raises(ValueError):
            p.load(other)
    with open(p.path) as f:
        st = json.load(f)
    st["version"] = 0
    with open(p.path, "w") as f:
        json.dump(st, f)
    with pytest.raises(ValueError):
        p.load(StreamConfig(seed=5, chunks=25))


def test_npz_sink(tmp_path):
    sink = NpzSink(str(tmp_path / "out"))
    idx = np.array([3, 9, 40], np.int64)
    paths = np.arange(3 * 4 * 2, dtype=np.float32).reshape(3, 4, 2)
    xf = np.ones((3, 5), np.float32)
    sink(7, idx, paths, xf)
    with np.load(sink.path_of(7)) as z:
        assert np.array_equal(z["index"], idx) and np.array_equal(z["paths"], paths)
        assert np.array_equal(z["xform"], xf)
    assert sorted(os.listdir(sink.out_dir)) == ["chunk_000007.npz"]
