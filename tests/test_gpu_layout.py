"""The blocked workspace layout's parameters (rows per block, block-stride pad,
column tile width) change where the intermediate lives, never the result:
the filter matches the FP64 oracle under every setting, and settings that
differ only in the pad give bit-identical outputs.  Also checks that the
workspace and saved-spectrum sizes cover the padded layout."""
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, announce, need_gpu, rel_l2, to_host

pytestmark = pytest.mark.gpu

_KNOBS = ("FFTMI_RB", "FFTMI_BLOCK_PAD", "FFTMI_COLS_W")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _filter_with(env, img, mask, flags_extra=0):
    """Run fft2d_filter through a plan created under the given layout knobs."""
    import torch
    from paper_cs_0103001_amd import _binding as B
    from paper_cs_0103001_amd import api
    saved = {k: os.environ.get(k) for k in _KNOBS}
    try:
        for k in _KNOBS:
            os.environ.pop(k, None)
        os.environ.update({k: str(v) for k, v in env.items()})
        x = torch.from_numpy(np.ascontiguousarray(img)).cuda()
        n, m = img.shape[-2:]
        batch = img.shape[0] if img.ndim == 3 else 1
        plan = api.Plan(2, (n, m), batch, B.FFT_IN_REAL_F32 | flags_extra, x.device)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    out = torch.empty(img.shape, dtype=torch.complex64, device=x.device)
    ws = plan.workspace()
    mk = B.make_mask(**mask)
    B.fft2d_filter(plan.h, api._ptr(x), api._ptr(out), mk, api._ptr(ws), api._stream(x.device))
    return to_host(out), plan


LAYOUTS = [dict(FFTMI_RB=rb, FFTMI_BLOCK_PAD=pad, FFTMI_COLS_W=w)
           for rb in (1, 2, 4, 8) for pad in (0, 32, 96) for w in (1, 2)]


@pytest.mark.parametrize("N,M", [(256, 256), (128, 512), (1024, 64)])
def test_layouts_match_oracle_and_each_other(N, M):
    img = np.stack([synth.star_field(N, M, 120, 1.5, seed=(31, N, M, b)) for b in range(2)])
    mask = dict(kind="butterworth", cutoff=0.15, order=4)
    ref = oracle.filter2(img, oracle.mask_butterworth(N, M, 0.15, 4))
    by_rb_w = {}
    for env in LAYOUTS:
        announce("layout %s %dx%d" % (env, N, M))
        got, plan = _filter_with(env, img, mask)
        assert rel_l2(got, ref, 2) < TOL, env
        key = (env["FFTMI_RB"], env["FFTMI_COLS_W"])
        if key in by_rb_w:
            # the pad moves data, not arithmetic
            assert np.array_equal(got, by_rb_w[key]), env
        else:
            by_rb_w[key] = got


def test_padded_sizes_cover_layout():
    """4096-wide rows with 4 rows per block: the block stride is padded by 32
    elements, and the workspace and saved spectrum grow accordingly."""
    from paper_cs_0103001_amd import _binding as B
    from paper_cs_0103001_amd import api
    import torch
    n, m, batch = 256, 4096, 3
    plan = api.Plan(2, (n, m), batch, B.FFT_IN_REAL_F32, torch.device("cuda", 0))
    blocked = batch * (n // 4) * (4 * m + 32) * 8
    # the saved spectrum, or the state of the frequency-domain MSE (row
    # spectra of x - c and per-bin sums), whichever is larger
    assert plan.spectrum_bytes >= blocked
    assert plan.workspace_bytes >= blocked


def test_full_size_4096_pad_variants():
    """The 4096^2 image (the headline workload) under the default pad and
    without it: identical outputs, both at the oracle's tolerance."""
    img = synth.image_4096(0)
    mask = dict(kind="butterworth", cutoff=0.15, order=4)
    announce("4096^2 pad 0")
    a, _ = _filter_with(dict(FFTMI_BLOCK_PAD=0), img, mask)
    announce("4096^2 pad 32")
    b, _ = _filter_with(dict(FFTMI_BLOCK_PAD=32), img, mask)
    assert np.array_equal(a, b)
    ref = oracle.filter2(img, oracle.mask_butterworth(4096, 4096, 0.15, 4))
    assert rel_l2(b, ref, 2) < TOL
