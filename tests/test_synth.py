"""The seeded input generators: deterministic per seed and independent of
the thread count; the fast 4:2:0 frame path equals the direct evaluation."""
import numpy as np

import synth


def test_plane_is_deterministic_and_thread_independent():
    a = synth.plane(200, 96, 42, threads=1)
    b = synth.plane(200, 96, 42, threads=7)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, synth.plane(200, 96, 43))
    assert a.dtype == np.uint8 and a.shape == (96, 200)


def test_batch_matches_single_planes():
    sizes = [(64, 32), (24, 8), (128, 72)]
    buf, off, strides = synth.batch(sizes, [5, 6, 7])
    for i, (w, h) in enumerate(sizes):
        assert np.array_equal(synth.batch_view(buf, off, strides, sizes, i), synth.plane(w, h, 5 + i))
        assert off[i] % 256 == 0


def test_video_canvas_path_equals_direct_evaluation():
    v = synth.Video420(w=320, h=240, frames=6, seed=9)
    for f in (0, 3, 5):
        fast = v.frame(f)
        slow = v.frame_direct(f)
        for a, b in zip(fast, slow):
            assert np.array_equal(a, b)
    assert v.frame(1)[0].shape == (240, 320) and v.frame(1)[1].shape == (120, 160)


def test_workload_specs():
    sizes, seeds, qs = synth.ragged_batch_spec(n=500)
    w = np.array([s[0] for s in sizes])
    h = np.array([s[1] for s in sizes])
    assert (w % 8 == 0).all() and (h % 8 == 0).all()
    assert w.min() >= 64 and w.max() <= 2048 and h.min() >= 64 and h.max() <= 2048
    for q in qs[:20]:
        s = int(q[0, 1]) - 1
        assert 1 <= s <= 8 and np.array_equal(q, synth.qtable(1, s))
    tr = synth.serving_trace(1000, 2.0, seed=5)
    assert abs(len(tr["t"]) - 2000) < 200
    assert (np.maximum(tr["w"], tr["h"]) <= 4 * np.minimum(tr["w"], tr["h"])).all()
    assert set(np.unique(tr["op"])) <= {0, 1} and tr["s"].min() >= 1 and tr["s"].max() <= 8
