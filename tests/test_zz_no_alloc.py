"""GPU: fl_analyze_noalloc, the entry point that allocates no device memory
(all its buffers live in the library's fixed scratch array), against
fl_analyze on the same inputs, through the C ABI."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2210_01465_amd import synth

pytestmark = pytest.mark.gpu
NB = {"hamming": 0, "adjacent": 1}


def say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2210_01465_amd import api
    c = api.Context(0)
    yield c
    c.close()


def _call(ctx, name, radix, fit, nb, bufs, d=0.85, p=0.05):
    """One fl_analyze / fl_analyze_noalloc call through the C ABI into the
    preallocated buffers; returns (status, summary, pagerank, minima, valid_raw)."""
    import torch
    from paper_2210_01465_amd import _abi
    pr, mins, vraw = bufs
    arr = (ctypes.c_int32 * len(radix))(*radix)
    sp = _abi.fl_space(len(radix), ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32)))
    prm = _abi.fl_params(d, p, 0.0, 0, 0)
    out = _abi.fl_summary()
    rc = getattr(_abi.load(), name)(ctx.handle, ctypes.byref(sp), ctypes.c_void_p(fit.data_ptr()), NB[nb],
                                    ctypes.byref(prm), ctypes.c_void_p(pr.data_ptr()),
                                    ctypes.c_void_p(mins.data_ptr()), ctypes.c_void_p(vraw.data_ptr()),
                                    ctypes.byref(out))
    torch.cuda.synchronize()
    if rc != 0:
        return rc, out, None, None, None
    N, M = int(out.n_valid), int(out.n_minima)
    return rc, out, pr[:N].cpu().numpy(), mins[:M].cpu().numpy(), vraw[:N].cpu().numpy()


def _buffers(n_raw):
    import torch
    return (torch.full((n_raw,), -1.0, dtype=torch.float64, device="cuda"),
            torch.full((n_raw,), -7, dtype=torch.int32, device="cuda"),
            torch.full((n_raw,), -7, dtype=torch.int32, device="cuda"))


def _same(ctx, space, nb, bufs, d=0.85):
    import torch
    fit = torch.from_numpy(np.ascontiguousarray(space.fitness_raw)).cuda()
    say(f"noalloc {space.name} radix={space.radix} nb={nb} d={d}")
    got = _call(ctx, "fl_analyze_noalloc", space.radix, fit, nb, bufs, d)
    ref = _call(ctx, "fl_analyze", space.radix, fit, nb, _buffers(space.n_raw), d)
    assert got[0] == 0 and ref[0] == 0, (got[0], ref[0], ctx_error(ctx))
    for f in ("n_raw", "n_valid", "n_edges", "n_minima", "iterations", "n_plateau", "row_mapping"):
        assert getattr(got[1], f) == getattr(ref[1], f), f
    assert got[1].score == ref[1].score and got[1].residual_l1 == ref[1].residual_l1
    assert np.array_equal(got[2], ref[2])          # ranks bit for bit
    assert np.array_equal(got[3], ref[3]) and np.array_equal(got[4], ref[4])
    a = oracle.analyze(space.radix, space.fitness_raw, NB[nb], d, 0.05, tol=1e-12)
    assert np.array_equal(got[3], a.graph.minima) and np.array_equal(got[4], a.graph.valid_raw)
    assert float(np.abs(got[2] - a.pagerank).sum()) <= 1e-5
    assert abs(got[1].score - a.score) <= 1e-5


def ctx_error(ctx):
    from paper_2210_01465_amd import api
    return api.last_error(ctx)


def test_noalloc_two_calls_second_smaller(ctx):
    """The mid workload (207 360 raw / 124 762 valid), then a tiny one in
    the same output buffers: each equals fl_analyze on the same input."""
    mid = synth.mid()
    bufs = _buffers(mid.n_raw)
    _same(ctx, mid, "hamming", bufs)
    _same(ctx, synth.tiny(3), "hamming", bufs)


def test_noalloc_layouts_and_neighbourhoods(ctx):
    """Adjacent neighbourhood, a space too wide for node records (CSR sweep
    and the generic build kernels), and one of the batched workload's
    largest spaces, back to back on the shared scratch array."""
    rng = np.random.default_rng(5)
    wide = synth.Space("wide", (200, 3), rng.lognormal(0.0, 0.5, 600).astype(np.float32))
    biggest = max(synth.batched(), key=lambda s: s.n_raw)
    bufs = _buffers(max(biggest.n_raw, 600))
    _same(ctx, synth.mid(), "adjacent", bufs, d=0.9)
    _same(ctx, wide, "hamming", bufs)
    _same(ctx, biggest, "hamming", bufs, d=0.8)
    _same(ctx, synth.tiny(1), "adjacent", bufs)


def test_noalloc_rejects_spaces_beyond_the_scratch(ctx):
    """A space whose raw size alone exceeds the scratch array is rejected
    before any launch; one that fits by raw size but whose FFG does not is
    rejected after the degree count; calls afterwards are unaffected."""
    import torch
    from paper_2210_01465_amd import _abi
    large = synth.large()                               # 4 665 600 raw configurations
    fit = torch.from_numpy(large.fitness_raw).cuda()
    say("noalloc rejects the large workload up front")
    rc = _call(ctx, "fl_analyze_noalloc", large.radix, fit, "hamming", _buffers(16))[0]
    assert rc == _abi.FL_EINVAL and "scratch" in ctx_error(ctx)
    radix = (16, 16, 16, 16, 12)                        # 786 432 raw: 15.7 MB, fits by raw size
    rng = np.random.default_rng(9)
    f = rng.lognormal(0.0, 0.5, int(np.prod(radix))).astype(np.float32)
    say(f"noalloc rejects radix={radix} after the degree count")
    fit = torch.from_numpy(f).cuda()
    rc = _call(ctx, "fl_analyze_noalloc", radix, fit, "hamming", _buffers(f.size))[0]
    assert rc == _abi.FL_EINVAL and "scratch" in ctx_error(ctx), ctx_error(ctx)
    _same(ctx, synth.tiny(2), "hamming", _buffers(160))
