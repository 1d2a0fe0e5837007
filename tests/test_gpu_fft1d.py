"""1D transforms on the GPU against the FP64 oracle (eq. E2 forward with 1/N,
eq. E3 inverse unscaled), every power-of-two length up to 2^22."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, announce, need_gpu, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _api():
    from paper_cs_0103001_amd import api
    return api


SINGLE = list(range(0, 15))          # one LDS pass
FOURSTEP = [15, 16, 17, 18, 20]       # two strided passes


@pytest.mark.parametrize("lg", SINGLE + FOURSTEP)
def test_forward_inverse_vs_oracle(lg):
    api = _api()
    n = 1 << lg
    batch = 5 if lg < 16 else 2        # 5 rows: the last workgroup is partly empty
    x = synth.uniform_complex((batch, n), (11, lg))
    announce("fft1d n=%d batch=%d" % (n, batch))
    X = to_host(api.fft(to_dev(x)))
    assert rel_l2(X, oracle.fft(x, threads=4), 1) < TOL
    announce("ifft1d n=%d batch=%d" % (n, batch))
    f = to_host(api.ifft(to_dev(x)))
    assert rel_l2(f, oracle.ifft(x, threads=4), 1) < TOL


@pytest.mark.parametrize("lg", [0, 3, 10, 12, 14, 16])
def test_norms_adjoints_and_real_io(lg):
    api = _api()
    from paper_cs_0103001_amd import _binding as B
    n = 1 << lg
    x = synth.uniform_complex((3, n), (12, lg))
    xd = to_dev(x)
    ref_f = oracle.fft(x, threads=4)
    ref_i = oracle.ifft(x, threads=4)
    announce("fft1d norms n=%d" % n)
    assert rel_l2(to_host(api.fft(xd, norm="numpy")), ref_f * n, 1) < TOL
    assert rel_l2(to_host(api.ifft(xd, norm="numpy")), ref_i / n, 1) < TOL
    # adjoint of the forward (1/N) F^H and of the inverse F
    assert rel_l2(to_host(api.transform(xd, 1, B.FFT_ADJ_FORWARD)), ref_i / n, 1) < TOL
    assert rel_l2(to_host(api.transform(xd, 1, B.FFT_ADJ_INVERSE)), ref_f * n, 1) < TOL
    if lg <= 14:
        xr = x.real.copy()
        assert rel_l2(to_host(api.fft(to_dev(xr))), oracle.fft(xr, threads=4), 1) < TOL
        got = to_host(api.ifft(xd, real_output=True))
        assert got.dtype == np.float32
        assert rel_l2(got, ref_i.real, 1) < TOL


def test_empty_batch():
    api = _api()
    import torch
    x = torch.empty((0, 256), dtype=torch.complex64, device="cuda")
    assert api.fft(x).shape == (0, 256)


@pytest.mark.parametrize("lg", [10, 14, 16, 22])
def test_full_sweep_batch_sampled_rows(lg):
    """The 256 MiB batch of the 1D sweep, in the launch shape the benchmark
    times; sampled rows are checked against the oracle, and the round trip
    against the input."""
    api = _api()
    n = 1 << lg
    batch = synth.sweep_1d_batch(lg)
    x = synth.sweep_1d(lg, batch)
    announce("fft1d sweep n=%d batch=%d" % (n, batch))
    xd = to_dev(x)
    X = api.fft(xd)
    back = api.ifft(X)
    rows = sorted({0, batch // 3, batch - 1})
    Xh = to_host(X[rows])
    assert rel_l2(Xh, oracle.fft(x[rows], threads=8), 1) < TOL
    assert rel_l2(to_host(back), x, 1) < TOL


def test_deterministic():
    api = _api()
    x = to_dev(synth.uniform_complex((64, 4096), 5))
    a = to_host(api.fft(x))
    b = to_host(api.fft(x))
    np.testing.assert_array_equal(a, b)


_FS_KNOBS = ("FFTMI_FS_PAD", "FFTMI_FS_W", "FFTMI_FS_THREADS1", "FFTMI_FS_THREADS2", "FFTMI_FS_LOG_N1", "FFTMI_FS_NT",
             "FFTMI_FS_NT1", "FFTMI_FS_CHUNK_MB")


def _fft_with(env, x, direction):
    """One fft_exec through a plan created under the given four-step knobs."""
    import os
    import torch
    from paper_cs_0103001_amd import _binding as B
    from paper_cs_0103001_amd import api
    saved = {k: os.environ.get(k) for k in _FS_KNOBS}
    try:
        for k in _FS_KNOBS:
            os.environ.pop(k, None)
        os.environ.update({k: str(v) for k, v in env.items()})
        plan = api.Plan(1, (x.shape[-1],), x.shape[0], 0, x.device)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    out = torch.empty_like(x)
    ws = plan.workspace()
    B.fft_exec(plan.h, api._ptr(x), api._ptr(out), api._ptr(ws), direction, api._stream(x.device))
    return to_host(out), plan


@pytest.mark.parametrize("lg", [15, 18, 21])
def test_fourstep_layout_knobs(lg):
    """The padded row stride of the four-step intermediate and the column tile
    width move data, not arithmetic: every setting matches the oracle, all
    outputs are bit-identical, and the workspace covers the padded rows."""
    from paper_cs_0103001_amd import _binding as B
    n = 1 << lg
    n1, n2 = 1 << (lg // 2), 1 << (lg - lg // 2)
    batch = 3
    x = synth.uniform_complex((batch, n), 40 + lg)
    xd = to_dev(x)
    ref = oracle.fft(x, threads=8)
    # bit-identical among the settings of one kernel build (threads per tile);
    # the 1024-thread build is another compilation of the transform, whose
    # floating-point contractions may differ in the last bit
    first = {}
    for pad, w, thr in [(p_, w_, 512) for p_ in (0, 32, 96) for w_ in (16, 4, 1)] + [(0, 16, 1024), (32, 16, 1024)]:
        env = dict(FFTMI_FS_PAD=pad, FFTMI_FS_W=w, FFTMI_FS_THREADS1=thr, FFTMI_FS_THREADS2=thr)
        announce("fft1d four-step n=2^%d %s" % (lg, env))
        got, plan = _fft_with(env, xd, B.FFT_FORWARD)
        assert plan.workspace_bytes >= batch * n2 * (n1 + pad) * 8, env
        assert rel_l2(got, ref, 1) < TOL, env
        if thr not in first:
            first[thr] = got
        else:
            assert np.array_equal(got, first[thr]), env
    if len(first) == 2:
        assert rel_l2(first[1024], first[512], 1) < 1e-6


@pytest.mark.parametrize("lg", [19, 20, 22])
def test_fourstep_wide_tiles(lg):
    """1024-thread four-step tiles (twice the columns per tile) against the
    oracle in both directions, and against the 512-thread tiles."""
    from paper_cs_0103001_amd import _binding as B
    x = synth.uniform_complex((2, 1 << lg), (14, lg))
    xd = to_dev(x)
    for direction, ref in ((B.FFT_FORWARD, oracle.fft(x, threads=8)), (B.FFT_INVERSE, oracle.ifft(x, threads=8))):
        outs = []
        for t1, t2 in ((512, 512), (512, 1024), (1024, 512), (1024, 1024)):
            announce("fft1d four-step n=2^%d dir %d threads %d/%d" % (lg, direction, t1, t2))
            got, plan = _fft_with(dict(FFTMI_FS_THREADS1=t1, FFTMI_FS_THREADS2=t2), xd, direction)
            assert rel_l2(got, ref, 1) < TOL
            outs.append(got)
        for o in outs[1:]:
            assert rel_l2(o, outs[0], 1) < 1e-6


@pytest.mark.parametrize("lg", [16, 20, 21])
def test_fourstep_nontemporal_hints(lg):
    """Pass two with none, either or both of its non-temporal loads and
    stores (stores by default up to 2^20 points), and pass one with and
    without its non-temporal input loads (taken by its 1024-thread tiles,
    2^21 here): cache hints only, so every combination is bit-identical and
    matches the oracle in both directions."""
    from paper_cs_0103001_amd import _binding as B
    x = synth.uniform_complex((2, 1 << lg), (16, lg))
    xd = to_dev(x)
    for direction, ref in ((B.FFT_FORWARD, oracle.fft(x, threads=8)), (B.FFT_INVERSE, oracle.ifft(x, threads=8))):
        outs = []
        for nt, nt1 in ((0, 0), (1, 0), (2, 0), (3, 0), (0, 1), (3, 1)):
            announce("fft1d four-step n=2^%d dir %d non-temporal pass two %d pass one %d" % (lg, direction, nt, nt1))
            got, _ = _fft_with(dict(FFTMI_FS_NT=nt, FFTMI_FS_NT1=nt1), xd, direction)
            assert rel_l2(got, ref, 1) < TOL, (nt, nt1)
            outs.append(got)
        for o in outs[1:]:
            assert np.array_equal(outs[0], o)


@pytest.mark.parametrize("lg", [16, 19, 21])
def test_fourstep_chunks(lg):
    """The batch in chunks of batch entries (each chunk's two passes reuse the
    start of the workspace, which holds one chunk), including a last chunk
    shorter than the others: bit-identical to the whole batch at once, and
    the oracle's result."""
    from paper_cs_0103001_amd import _binding as B
    batch = 5
    x = synth.uniform_complex((batch, 1 << lg), (17, lg))
    xd = to_dev(x)
    per_entry_mib = (1 << lg) * 8 / float(1 << 20)
    for direction, ref in ((B.FFT_FORWARD, oracle.fft(x, threads=8)), (B.FFT_INVERSE, oracle.ifft(x, threads=8))):
        outs, ws = [], []
        for mib in (0, int(2 * per_entry_mib) + 1, 128):  # whole batch, chunks of 2-4 entries, default
            announce("fft1d four-step n=2^%d batch %d chunk %d MiB dir %d" % (lg, batch, mib, direction))
            got, plan = _fft_with(dict(FFTMI_FS_CHUNK_MB=mib), xd, direction)
            assert rel_l2(got, ref, 1) < TOL, (mib, direction)
            outs.append(got)
            ws.append(B.fft_workspace_size(plan.h))
        for o in outs[1:]:
            assert np.array_equal(o, outs[0])
        # the workspace holds one chunk: a whole number of the entries of the
        # whole-batch plan's, fewer of them for the smaller chunks
        per_entry = ws[0] // batch
        assert ws[0] == per_entry * batch and per_entry >= (1 << lg) * 8
        assert ws[1] % per_entry == 0 and ws[1] < ws[0]
        assert ws[2] % per_entry == 0 and ws[2] <= ws[0]


@pytest.mark.parametrize("lg", [15, 20, 22])
def test_fourstep_uneven_splits(lg):
    """Every split N = N1 N2 with both lengths in 2^7 .. 2^12, one plan after
    another in one process (each split has its own table of W_N^{k1 n2}),
    forward and inverse against the oracle."""
    from paper_cs_0103001_amd import _binding as B
    x = synth.uniform_complex((2, 1 << lg), (15, lg))
    xd = to_dev(x)
    refs = {B.FFT_FORWARD: oracle.fft(x, threads=8), B.FFT_INVERSE: oracle.ifft(x, threads=8)}
    for n1 in range(max(7, lg - 12), min(12, lg - 7) + 1):
        for direction, ref in refs.items():
            announce("fft1d four-step n=2^%d split 2^%d x 2^%d dir %d" % (lg, n1, lg - n1, direction))
            got, plan = _fft_with(dict(FFTMI_FS_LOG_N1=n1), xd, direction)
            assert plan.workspace_bytes >= 2 * (1 << lg) * 8
            assert rel_l2(got, ref, 1) < TOL, (n1, direction)


@pytest.mark.parametrize("lg", [23, 24])
def test_longest_lengths_vs_oracle(lg):
    """The two lengths above the measured sweep that the plan accepts (2^23:
    2^11 x 2^12 split, 2^24: 4096-point strided columns in both passes),
    forward and inverse against the FP64 oracle."""
    api = _api()
    n = 1 << lg
    x = synth.uniform_complex((2, n), (13, lg))
    announce("fft1d n=2^%d batch=2" % lg)
    X = to_host(api.fft(to_dev(x)))
    ef = rel_l2(X, oracle.fft(x, threads=8), 1)
    announce("ifft1d n=2^%d batch=2" % lg)
    f = to_host(api.ifft(to_dev(x)))
    ei = rel_l2(f, oracle.ifft(x, threads=8), 1)
    print("2^%d forward relL2 %.3e inverse %.3e" % (lg, ef, ei))
    assert ef < TOL and ei < TOL
