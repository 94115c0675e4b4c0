"""Host-side pieces of the serving form (no GPU): the request stream's composition and the
server entry points' argument checks."""
import ctypes

import numpy as np

from paper_1406_0359_amd import purify, synth


def test_size_mix_is_8_4_2_1_by_largest_remainder():
    assert synth.serving_counts(512) == [273, 137, 68, 34]
    assert synth.serving_counts(30) == [16, 8, 4, 2]
    for c in (1, 7, 15, 100, 511):
        per = synth.serving_counts(c)
        assert sum(per) == c and all(p >= 0 for p in per)


def test_requests_are_seeded_and_within_the_stated_ranges():
    a, b = synth.serving_requests(15), synth.serving_requests(15)
    sizes = [p.x_true.shape[0] for p in a]
    assert sorted(sizes) == sorted([128] * 8 + [256] * 4 + [512] * 2 + [1024])
    for p, q in zip(a, b):
        n = p.x_true.shape[0]
        assert np.array_equal(p.uv, q.uv) and np.array_equal(p.x_true, q.x_true)
        assert 0.2 * n * n - 1 <= p.uv.shape[0] <= 2.0 * n * n + 1
        assert 20.0 <= p.extra["isnr_db"] <= 40.0
        assert np.all(np.abs(p.uv) <= np.pi) and p.x_true.min() >= 0


def test_poisson_arrivals_have_the_requested_rate():
    t = synth.poisson_arrivals(20000, 5.0)
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    assert abs(np.mean(np.diff(t)) - 0.2) < 0.01


def test_server_rejects_bad_descriptors_without_touching_the_device():
    lib = purify.load_library()
    h = ctypes.c_void_p()
    d = purify.ServerDesc()
    d.arena, d.arena_bytes, d.max_active = None, 1 << 20, 2
    assert lib.purify_server_create(ctypes.byref(d), ctypes.byref(h)) == 1
    d.arena, d.max_active = 4096, 0
    assert lib.purify_server_create(ctypes.byref(d), ctypes.byref(h)) == 1
    d.arena, d.max_active = 4097, 2            # not 256-byte aligned
    assert lib.purify_server_create(ctypes.byref(d), ctypes.byref(h)) == 1
    assert lib.purify_server_poll(None, 1) == -1
