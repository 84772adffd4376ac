"""The chunked stream on the GPU: each chunk equals a direct generate, simulate and
normalise call over the same candidates; a stream stopped part way and resumed
from its progress file delivers exactly the chunks of an uninterrupted run, and a
chunk delivered again (its progress entry lost) has the same contents."""
import json
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_14567_amd import links
    return links


class Collect:
    def __init__(self):
        self.got = {}
        self.order = []

    def __call__(self, c, index, paths, xform):
        self.got[c] = (index.copy(), paths.copy(), xform.copy())
        self.order.append(c)


def _same(a, b):
    return all(np.array_equal(x, y, equal_nan=True) for x, y in zip(a, b))


def test_stream_chunks_and_resume(L, tmp_path):
    from paper_2208_14567_amd import stream as S
    cfg = S.StreamConfig(seed=21, chunks=5, chunk=20000, cap=20000, rules=True, n_lo=5, n_hi=20)
    _say(f"[stream] {cfg}")
    full = Collect()
    tot = S.Streamer(cfg).run(sink=full)
    assert full.order == [0, 1, 2, 3, 4]
    assert tot["candidates"] == 100000 and tot["next_chunk"] == 5 and tot["dropped"] == 0
    assert tot["valid"] == sum(len(v[0]) for v in full.got.values()) > 0

    # chunk 3 against a direct call over the same candidates
    ctx = L.Context(0)
    db = ctx.generate_dyads(cfg.chunk, cfg.seed, first=3 * cfg.chunk, n_lo=cfg.n_lo, n_hi=cfg.n_hi, rules=True)
    r = ctx.simulate(db, T=cfg.T, write=L.WRITE_VALID, cap=cfg.cap)
    norm, xf = ctx.normalize_paths_n(r["path"], r["n_written"], L.NORM_PCA)
    k = int(r["n_written"].cpu()[0])
    want = (r["path_index"][:k].cpu().numpy().astype(np.int64) + 3 * cfg.chunk, norm[:k].cpu().numpy(),
            xf[:k].cpu().numpy())
    assert _same(full.got[3], want)

    # stopped after two chunks, resumed by a new streamer from the progress file
    prog = str(tmp_path / "progress.json")
    first = Collect()
    t1 = S.Streamer(cfg).run(sink=first, progress_path=prog, max_chunks=2)
    assert first.order == [0, 1] and t1["next_chunk"] == 2
    with open(prog) as f:
        assert json.load(f)["next_chunk"] == 2
    rest = Collect()
    t2 = S.Streamer(cfg).run(sink=rest, progress_path=prog)
    assert rest.order == [2, 3, 4]
    for c in range(5):
        assert _same((first.got | rest.got)[c], full.got[c])
    assert t2["valid"] == tot["valid"] and t2["candidates"] == tot["candidates"]

    # the progress entry of chunk 4 lost: chunk 4 is delivered again, the same
    with open(prog) as f:
        st = json.load(f)
    st["next_chunk"] = 4
    with open(prog, "w") as f:
        json.dump(st, f)
    again = Collect()
    S.Streamer(cfg).run(sink=again, progress_path=prog)
    assert again.order == [4] and _same(again.got[4], full.got[4])

    # files written by the chunk sink hold the same arrays
    sink = S.NpzSink(str(tmp_path / "out"))
    S.Streamer(cfg).run(sink=sink, max_chunks=2)
    with np.load(sink.path_of(1)) as z:
        assert _same((z["index"], z["paths"], z["xform"]), full.got[1])

    with pytest.raises(ValueError):
        S.Streamer(S.StreamConfig(seed=22, chunks=5, chunk=20000, cap=20000)).run(progress_path=prog)
    _say(f"  {tot['valid']} valid of {tot['candidates']}; resumed run equal chunk for chunk")


def test_stream_cap_drops_the_rest(L):
    from paper_2208_14567_amd import stream as S
    cfg = S.StreamConfig(seed=23, chunks=2, chunk=20000, cap=100)
    c = Collect()
    tot = S.Streamer(cfg).run(sink=c)
    assert all(len(v[0]) == 100 for v in c.got.values())
    assert tot["dropped"] == tot["valid"] - 200 > 0


def test_stream_inspect_strided_statuses(L):
    from paper_2208_14567_amd import stream as S
    cfg = S.StreamConfig(seed=24, chunks=3, chunk=20000, cap=20000)
    seen = {}

    def inspect(c, status, fail_step):
        seen[c] = (status.copy(), fail_step.copy())

    # 20000 / 7 rounds up to 2858 candidates per chunk; the keep is capped there
    S.Streamer(cfg, keep_status=5000, status_stride=7).run(inspect=inspect)
    assert sorted(seen) == [0, 1, 2]
    ctx = L.Context(0)
    db = ctx.generate_dyads(cfg.chunk, cfg.seed, first=2 * cfg.chunk)
    r = ctx.simulate(db, T=cfg.T, write=L.WRITE_VALID, cap=cfg.cap)
    st, fs = seen[2]
    assert len(st) == 2858
    assert np.array_equal(st, r["status"].cpu().numpy()[::7])
    assert np.array_equal(fs, r["fail_step"].cpu().numpy()[::7])
    with pytest.raises(ValueError):
        S.Streamer(cfg, keep_status=10, status_stride=0)


@pytest.mark.parametrize("x0_f32", [False, True])
def test_stream_from_host_batch(L, x0_f32):
    """A stream fed from a batch in host memory (chunks copied from pinned memory
    on each lane's stream) delivers the same chunks as the stream that generates
    the same candidates on the device, with positions crossing in double or
    (exact here) single precision."""
    from paper_2208_14567_amd import gen
    from paper_2208_14567_amd import stream as S
    cfg = S.StreamConfig(seed=25, chunks=3, chunk=20000, cap=20000)
    host = gen.dyad_batch(cfg.chunks * cfg.chunk, cfg.seed, gen.n_uniform(cfg.n_lo, cfg.n_hi), cfg.J)
    dev, fed = Collect(), Collect()
    S.Streamer(cfg).run(sink=dev)
    tot = S.Streamer(cfg, host=host, x0_f32=x0_f32).run(sink=fed)
    assert fed.order == [0, 1, 2]
    for c in range(3):
        assert _same(fed.got[c], dev.got[c]), c
    per = cfg.chunk * (1 + 4 * cfg.J + 4 + 2 + cfg.J * 2 * (4 if x0_f32 else 8))
    assert tot["h2d_bytes"] == 3 * per
    with pytest.raises(ValueError):
        S.Streamer(cfg, host=host.slice(0, 1000))
    if x0_f32:
        bad = host.slice(0, cfg.chunks * cfg.chunk)
        bad.x0 = bad.x0 + 1e-9
        with pytest.raises(ValueError):
            S.Streamer(cfg, host=bad, x0_f32=True)
