"""Ragged batches (mixed power-of-two sides in one persistent launch per
pass, captured in a HIP graph, autotuned schedule) against the FP64 oracle,
image by image."""
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, announce, need_gpu, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

SIGMA_F = 0.1


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _split(flat, sizes):
    out, off = [], 0
    for s in sizes:
        out.append(flat[off:off + s * s].reshape(s, s))
        off += s * s
    return out


def _check(got_flat, imgs, sizes, mask_kind="gaussian"):
    worst = 0.0
    for g, im, s in zip(_split(got_flat, sizes), imgs, sizes):
        if mask_kind == "gaussian":
            m = oracle.mask_gaussian(s, s, SIGMA_F)
        elif mask_kind == "butterworth":
            m = oracle.mask_butterworth(s, s, 0.15, 4)
        else:
            m = np.ones((s, s))
        ref = oracle.filter2(im, m, threads=4)
        err = rel_l2(g, ref, 2)
        worst = max(worst, err)
        assert err < TOL, (s, err)
    return worst


def _images(sizes, seed0=100, complex_input=False):
    imgs = [synth.ragged_image(seed0 + i, s) for i, s in enumerate(sizes)]
    if complex_input:
        rng = np.random.default_rng(seed0)
        imgs = [(im + 1j * rng.standard_normal(im.shape).astype(np.float32)).astype(np.complex64) for im in imgs]
    return imgs, np.concatenate([im.reshape(-1) for im in imgs])


MIXED = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 64, 8, 256, 1]


@pytest.mark.parametrize("kind", ["gaussian", "butterworth", "none"])
def test_ragged_mixed_sides_vs_oracle(kind):
    from paper_cs_0103001_amd import api
    imgs, flat = _images(MIXED)
    mask = {"gaussian": dict(kind="gaussian", sigma_f=SIGMA_F),
            "butterworth": dict(kind="butterworth", cutoff=0.15, order=4), "none": None}[kind]
    announce("ragged mixed %s" % kind)
    out = api.filter_ragged(to_dev(flat), MIXED, mask)
    print("worst relL2 %.3e" % _check(to_host(out), imgs, MIXED, kind))


def test_ragged_complex_in_real_out():
    from paper_cs_0103001_amd import api
    sizes = [64, 16, 256, 2, 128]
    imgs, flat = _images(sizes, seed0=200, complex_input=True)
    announce("ragged complex in")
    out = to_host(api.filter_ragged(to_dev(flat), sizes, dict(kind="gaussian", sigma_f=SIGMA_F)))
    _check(out, imgs, sizes)
    announce("ragged real out")
    imgs_r, flat_r = _images(sizes, seed0=300)
    outr = to_host(api.filter_ragged(to_dev(flat_r), sizes, dict(kind="gaussian", sigma_f=SIGMA_F),
                                     real_output=True))
    for g, im, s in zip(_split(outr, sizes), imgs_r, sizes):
        ref = oracle.filter2(im, oracle.mask_gaussian(s, s, SIGMA_F), threads=4).real
        assert rel_l2(g, ref, 2) < TOL


def test_ragged_graph_replays_match_eager():
    """The captured graph, replayed several times with other work and
    synchronisations in between, gives the eager launches' bits every time;
    a call with another output buffer captures again."""
    import torch
    from paper_cs_0103001_amd import _binding as B
    import ctypes
    sizes = [128, 2048, 64, 512, 256, 1024, 64]
    imgs, flat = _images(sizes, seed0=400)
    x = to_dev(flat)
    mk = B.make_mask("gaussian", sigma_f=SIGMA_F)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    outs = []
    for graph in ("0", "1"):
        os.environ["FFTMI_RAGGED_GRAPH"] = graph
        try:
            h = B.fft_plan_ragged(sizes, B.FFT_IN_REAL_F32)
        finally:
            os.environ.pop("FFTMI_RAGGED_GRAPH", None)
        ws = torch.empty(B.fft_workspace_size(h), dtype=torch.uint8, device="cuda")
        for rep in range(3):
            out = torch.full((x.numel(),), float("nan"), dtype=torch.complex64, device="cuda")
            if rep == 2:
                out2 = torch.empty_like(out)
                B.fft2d_filter_ragged(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out2.data_ptr()), mk,
                                      ctypes.c_void_p(ws.data_ptr()), st)
                outs.append(to_host(out2))
            announce("ragged graph=%s rep %d" % (graph, rep))
            B.fft2d_filter_ragged(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), mk,
                                  ctypes.c_void_p(ws.data_ptr()), st)
            torch.cuda.synchronize()
            _ = (torch.ones(1 << 20, device="cuda") * 3).sum().item()  # eager work between replays
            outs.append(to_host(out))
        B.fft_plan_destroy(h)
    _check(outs[0], imgs, sizes)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_ragged_autotune_keeps_results():
    from paper_cs_0103001_amd import api
    sizes = [2048, 64, 64, 128, 1024, 256, 512, 64]
    imgs, flat = _images(sizes, seed0=500)
    x = to_dev(flat)
    mask = dict(kind="gaussian", sigma_f=SIGMA_F)
    announce("ragged tune")
    sched = api.tune_ragged(x, sizes, mask)
    print("schedule", sched)
    assert sched["block"] in (256, 512) and sched["wg_cap"] in (0, 2)
    assert sched["chunk_bytes"] in (0, 128 << 20)
    _check(to_host(api.filter_ragged(x, sizes, mask)), imgs, sizes)


def test_ragged_workload_512_sampled():
    """The 512-image workload (sides uniform from {64..2048}, seed 3) at full
    size: every image finite and two runs bit-identical; two images of each
    side against the oracle."""
    from paper_cs_0103001_amd import api
    sizes = synth.ragged_sizes()
    announce("ragged 512: generating %d images" % len(sizes))
    flat = synth.ragged_batch(sizes, workers=min(16, os.cpu_count() or 1))
    x = to_dev(flat)
    mask = dict(kind="gaussian", sigma_f=SIGMA_F)
    announce("ragged 512: filter")
    out1 = api.filter_ragged(x, sizes, mask)
    out2 = api.filter_ragged(x, sizes, mask)
    a, b = to_host(out1), to_host(out2)
    assert np.isfinite(a.view(np.float32)).all()
    assert np.array_equal(a, b)
    offs = np.concatenate([[0], np.cumsum([s * s for s in sizes])])
    picked = []
    for side in sorted(set(sizes)):
        idx = [i for i, s in enumerate(sizes) if s == side][:2]
        picked += idx
    for i in picked:
        s = sizes[i]
        im = flat[offs[i]:offs[i + 1]].reshape(s, s)
        ref = oracle.filter2(im, oracle.mask_gaussian(s, s, SIGMA_F), threads=8)
        err = rel_l2(a[offs[i]:offs[i + 1]].reshape(s, s), ref, 2)
        assert err < TOL, (i, s, err)


def test_misaligned_workspace_rejected():
    """The kernels store 16-byte vectors into the workspace: a workspace
    pointer off a 16-byte boundary is refused with FFT_ERR_ARG before any
    launch, by the uniform, 1D and ragged entry points alike."""
    import ctypes
    import torch
    from paper_cs_0103001_amd import _binding as B
    from paper_cs_0103001_amd import api
    dev = torch.device("cuda", 0)
    st = api._stream(dev)
    mk = B.make_mask(kind="gaussian", sigma_f=SIGMA_F)

    def refused(call, ws):
        bad = ctypes.c_void_p(ws.data_ptr() + 8)
        with pytest.raises(B.FFTError) as ei:
            call(bad)
        assert ei.value.code == B.FFT_ERR_ARG

    x = torch.zeros((64, 64), dtype=torch.float32, device=dev)
    o = torch.empty((64, 64), dtype=torch.complex64, device=dev)
    p2 = api.Plan(2, (64, 64), 1, B.FFT_IN_REAL_F32, dev)
    ws2 = torch.empty(p2.workspace_bytes + 64, dtype=torch.uint8, device=dev)
    refused(lambda w: B.fft2d_filter(p2.h, api._ptr(x), api._ptr(o), mk, w, st), ws2)
    xc = torch.zeros((3, 1 << 15), dtype=torch.complex64, device=dev)
    oc = torch.empty_like(xc)
    p1 = api.Plan(1, (1 << 15,), 3, 0, dev)
    ws1 = torch.empty(p1.workspace_bytes + 64, dtype=torch.uint8, device=dev)
    refused(lambda w: B.fft_exec(p1.h, api._ptr(xc), api._ptr(oc), w, B.FFT_FORWARD, st), ws1)
    sizes = [64, 32, 1]
    xr = torch.zeros(sum(s * s for s in sizes), dtype=torch.float32, device=dev)
    orr = torch.empty(xr.numel(), dtype=torch.complex64, device=dev)
    pr = api.get_plan(0, (), len(sizes), B.FFT_IN_REAL_F32, dev, ragged_sizes=sizes)
    wsr = torch.empty(pr.workspace_bytes + 64, dtype=torch.uint8, device=dev)
    refused(lambda w: B.fft2d_filter_ragged(pr.h, api._ptr(xr), api._ptr(orr), mk, w, st), wsr)


def test_tune_cache_records_are_validated(tmp_path, monkeypatch):
    """A schedule the launchers would refuse is ignored at plan creation (the
    plan keeps the default schedule and runs); a valid record is adopted."""
    from paper_cs_0103001_amd import api
    from paper_cs_0103001_amd import _binding as B
    sizes = [256, 64, 128, 64]
    imgs, flat = _images(sizes, seed0=700)
    x = to_dev(flat)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("FFTMI_TUNE_CACHE", str(cache))
    mask = dict(kind="gaussian", sigma_f=SIGMA_F)
    announce("tune cache validation")
    api.tune_ragged(x, sizes, mask)
    key = cache.read_text().split()[0]
    default = {"block": 256, "wg_cap": 0, "chunk_bytes": 0, "order": 0, "small_side": 128}
    for bad in ("7 0 0 0 7", "256 -1 0 0 7", "256 0 -5 0 7", "256 0 0 9 7", "512 0 0 0 7 extra", "256 0",
                "256 0 0 0 8", "256 0 0 0 -2", "512 2 0 1"):
        cache.write_text("%s %s\n" % (key, bad))
        h = B.fft_plan_ragged(sizes, B.FFT_IN_REAL_F32)
        try:
            assert B.fft_plan_schedule(h) == default, bad
        finally:
            B.fft_plan_destroy(h)
    cache.write_text("%s 512 2 0 1 6\n" % key)
    h = B.fft_plan_ragged(sizes, B.FFT_IN_REAL_F32)
    try:
        assert B.fft_plan_schedule(h) == {"block": 512, "wg_cap": 2, "chunk_bytes": 0, "order": 1, "small_side": 64}
    finally:
        B.fft_plan_destroy(h)
    monkeypatch.delenv("FFTMI_TUNE_CACHE")
    _check(to_host(api.filter_ragged(x, sizes, mask)), imgs, sizes)


@pytest.mark.parametrize("small", [-1, 5, 7])
def test_ragged_single_pass_limit(small, monkeypatch):
    """Every side with the single-pass LDS path off, up to 32 and up to 128
    (FFTMI_RAGGED_SMALL, log2 of the largest such side): each image against
    the oracle, with real and complex input, c64 and f32 output, and a batch
    with more images of one side than a work item holds (64^2: 4 per item,
    32^2: 16), graph replays and eager launches alike."""
    from paper_cs_0103001_amd import _binding as B
    from paper_cs_0103001_amd import api
    import torch
    monkeypatch.setenv("FFTMI_RAGGED_SMALL", str(small))
    sizes = [128, 64, 64, 64, 64, 64, 32] * 3 + [32] * 14 + [16, 8, 4, 2, 1, 256, 512, 128, 1]
    for cplx, real_out in ((False, False), (True, True)):
        imgs, flat = _images(sizes, seed0=900 + small, complex_input=cplx)
        x = to_dev(flat)
        flags = (0 if cplx else B.FFT_IN_REAL_F32) | (B.FFT_OUT_REAL_F32 if real_out else 0)
        for graph in ("1", "0"):
            monkeypatch.setenv("FFTMI_RAGGED_GRAPH", graph)
            h = B.fft_plan_ragged(sizes, flags)
            try:
                sched = B.fft_plan_schedule(h)
                assert sched["small_side"] == (0 if small < 0 else 1 << small)
                out = torch.empty(x.numel(), dtype=torch.float32 if real_out else torch.complex64, device="cuda")
                ws = torch.empty(max(B.fft_workspace_size(h), 16), dtype=torch.uint8, device="cuda")
                mk = B.make_mask("butterworth", cutoff=0.15, order=4)
                announce("ragged single-pass limit %d complex %s graph %s" % (small, cplx, graph))
                for _ in range(2):
                    B.fft2d_filter_ragged(h, api._ptr(x), api._ptr(out), mk, api._ptr(ws), api._stream(x.device))
                got = to_host(out)
                for g, im, s in zip(_split(got, sizes), imgs, sizes):
                    ref = oracle.filter2(im, oracle.mask_butterworth(s, s, 0.15, 4), threads=4)
                    assert rel_l2(g, ref.real if real_out else ref, 2) < TOL, (s, small)
            finally:
                B.fft_plan_destroy(h)
