"""ctypes binding of libfftmi's C-ABI (include/fftmi.h): same names, argument
marshalling only.  Loading fails loudly when the HIP library is missing; there
is no CPU fallback."""
import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfftmi.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "fftmi.h")

FFT_OK = 0
FFT_ERR_ARG = -1
FFT_ERR_SIZE = -2
FFT_ERR_UNSUPPORTED = -3
FFT_ERR_WORKSPACE = -4
FFT_ERR_HIP = -5
FFT_ERR_NOMEM = -6
FFT_ERR_STATE = -7
FFT_ERR_SCRATCH = -8
FFT_NOALLOC_SCRATCH_BYTES = 144 << 20

FFT_FORWARD = -1
FFT_INVERSE = 1
FFT_ADJ_FORWARD = -2
FFT_ADJ_INVERSE = 2

FFT_IN_C64 = 0x0
FFT_IN_REAL_F32 = 0x1
FFT_OUT_C64 = 0x0
FFT_OUT_REAL_F32 = 0x2
FFT_NORM_PAPER = 0x0
FFT_NORM_NUMPY = 0x4
FFT_REAL_EVEN = 0x8

FFT_MASK_NONE = 0
FFT_MASK_TENSOR_F32 = 1
FFT_MASK_GAUSSIAN = 2
FFT_MASK_BUTTERWORTH = 3
FFT_MASK_DISC = 4


class fft_mask(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("data", ctypes.c_void_p), ("sigma_f", ctypes.c_double),
                ("cutoff", ctypes.c_double), ("order", ctypes.c_int), ("b", ctypes.c_double),
                ("c1", ctypes.c_double), ("c2", ctypes.c_double)]


class FFTError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__("%s: %s (status %d)" % (where, strerror(code), code))


_lib = None
_P = ctypes.c_void_p
_I64P = ctypes.POINTER(ctypes.c_int64)
_SIZEP = ctypes.POINTER(ctypes.c_size_t)
_MASKP = ctypes.POINTER(fft_mask)

_SIGS = {
    "fft_plan": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _I64P, ctypes.c_int64, ctypes.c_uint32]),
    "fft_workspace_size": (ctypes.c_int, [_P, _SIZEP]),
    "fft_spectrum_size": (ctypes.c_int, [_P, _SIZEP]),
    "fft_exec": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int, _P]),
    "fft2d_filter": (ctypes.c_int, [_P, _P, _P, _MASKP, _P, _P]),
    "fft2d_filter_noalloc": (ctypes.c_int, [_P, _P, _P, _MASKP, _P]),
    "fft2d_filter_stage": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _MASKP, _P, _P]),
    "fft2d_filter_save": (ctypes.c_int, [_P, _P, _P, _MASKP, _P, _P, _P]),
    "fft2d_filter_mask_grad": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "fft2d_filter_mse_grad": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_float, _P, _P, _P]),
    "fft2d_filter_mse": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_float, _P, _P, _P, _P]),
    "fft2d_filter_mse_spectral": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_float, _P, _P, _P, _P]),
    "fft2d_filter_mse_spectral_grad": (ctypes.c_int, [_P, _P, _P, ctypes.c_float, _P, _P]),
    "fft_plan_ragged": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int64, _I64P, ctypes.c_uint32]),
    "fft2d_filter_ragged": (ctypes.c_int, [_P, _P, _P, _MASKP, _P, _P]),
    "fft_plan_tune": (ctypes.c_int, [_P, _P, _P, _MASKP, _P, _P]),
    "fft_plan_schedule": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                         _I64P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "fft_plan_padded": (ctypes.c_int, [ctypes.POINTER(_P), _I64P, ctypes.c_int64, ctypes.c_uint32]),
    "fft2d_spectrum": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "fft_plan_layout": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), _I64P,
                                       ctypes.POINTER(ctypes.c_int)]),
    "fft_plan_tree": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int64, ctypes.c_int, ctypes.c_uint32]),
    "fft_tree_exec": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int64, _P]),
    "fft_plan_destroy": (ctypes.c_int, [_P]),
    "fft_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "fft_version": (ctypes.c_int, []),
}


def header_functions():
    """Names of the functions include/fftmi.h declares."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(fft\w+)\s*\(", text, flags=re.M)))


def lib():
    """The loaded libfftmi (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libfftmi.so is not built (%s); run __graft_entry__.build() or "
                              "python paper_cs_0103001_amd/build.py" % LIB_PATH)
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _lib = l
    return _lib


def strerror(code):
    return lib().fft_strerror(int(code)).decode()


def check(code, where):
    if code != FFT_OK:
        raise FFTError(code, where)


def _dims(dims):
    arr = (ctypes.c_int64 * len(dims))(*[int(d) for d in dims])
    return arr


def fft_plan(rank, dims, batch, flags=0):
    h = _P()
    check(lib().fft_plan(ctypes.byref(h), int(rank), _dims(dims), int(batch), int(flags)), "fft_plan")
    return h


def fft_plan_padded(dims0, batch, flags=0):
    h = _P()
    check(lib().fft_plan_padded(ctypes.byref(h), _dims(dims0), int(batch), int(flags)), "fft_plan_padded")
    return h


def fft2d_spectrum(plan, inp, magnitude, workspace, stream):
    check(lib().fft2d_spectrum(plan, inp, magnitude, workspace, stream), "fft2d_spectrum")


def fft_plan_ragged(sizes, flags=0):
    h = _P()
    check(lib().fft_plan_ragged(ctypes.byref(h), len(sizes), _dims(sizes), int(flags)), "fft_plan_ragged")
    return h


def fft_workspace_size(plan):
    n = ctypes.c_size_t(0)
    check(lib().fft_workspace_size(plan, ctypes.byref(n)), "fft_workspace_size")
    return n.value


def fft_spectrum_size(plan):
    n = ctypes.c_size_t(0)
    check(lib().fft_spectrum_size(plan, ctypes.byref(n)), "fft_spectrum_size")
    return n.value


def fft_exec(plan, inp, out, workspace, direction, stream):
    check(lib().fft_exec(plan, inp, out, workspace, int(direction), stream), "fft_exec")


def fft2d_filter(plan, inp, out, mask, workspace, stream):
    check(lib().fft2d_filter(plan, inp, out, ctypes.byref(mask) if mask is not None else None, workspace,
                             stream), "fft2d_filter")


def fft2d_filter_noalloc(plan, inp, out, mask, stream):
    check(lib().fft2d_filter_noalloc(plan, inp, out, ctypes.byref(mask) if mask is not None else None, stream),
          "fft2d_filter_noalloc")


def fft2d_filter_stage(plan, stage, inp, out, mask, workspace, stream):
    check(lib().fft2d_filter_stage(plan, int(stage), inp, out, ctypes.byref(mask) if mask is not None else None,
                                   workspace, stream), "fft2d_filter_stage")


def fft2d_filter_save(plan, inp, out, mask, spectrum, workspace, stream):
    check(lib().fft2d_filter_save(plan, inp, out, ctypes.byref(mask) if mask is not None else None, spectrum,
                                  workspace, stream), "fft2d_filter_save")


def fft2d_filter_mask_grad(plan, grad_y, spectrum, grad_mask, workspace, stream):
    check(lib().fft2d_filter_mask_grad(plan, grad_y, spectrum, grad_mask, workspace, stream),
          "fft2d_filter_mask_grad")


def fft2d_filter_mse_grad(plan, x, c, spectrum, mask, weight, grad_mask, workspace, stream):
    check(lib().fft2d_filter_mse_grad(plan, x, c, spectrum, mask, float(weight), grad_mask, workspace, stream),
          "fft2d_filter_mse_grad")


def fft2d_filter_mse(plan, x, c, mask, weight, spectrum, loss, workspace, stream):
    check(lib().fft2d_filter_mse(plan, x, c, mask, float(weight), spectrum, loss, workspace, stream),
          "fft2d_filter_mse")


def fft2d_filter_mse_spectral(plan, x, c, mask, weight, state, loss, workspace, stream):
    check(lib().fft2d_filter_mse_spectral(plan, x, c, mask, float(weight), state, loss, workspace, stream),
          "fft2d_filter_mse_spectral")


def fft2d_filter_mse_spectral_grad(plan, state, mask, weight, grad_mask, stream):
    check(lib().fft2d_filter_mse_spectral_grad(plan, state, mask, float(weight), grad_mask, stream),
          "fft2d_filter_mse_spectral_grad")


def fft2d_filter_ragged(plan, inp, out, mask, workspace, stream):
    check(lib().fft2d_filter_ragged(plan, inp, out, ctypes.byref(mask) if mask is not None else None, workspace,
                                    stream), "fft2d_filter_ragged")


def fft_plan_tune(plan, inp, out, mask, workspace, stream):
    check(lib().fft_plan_tune(plan, inp, out, ctypes.byref(mask) if mask is not None else None, workspace, stream),
          "fft_plan_tune")


def fft_plan_schedule(plan):
    b, c, o, sm = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    ch = ctypes.c_int64()
    check(lib().fft_plan_schedule(plan, ctypes.byref(b), ctypes.byref(c), ctypes.byref(ch), ctypes.byref(o),
                                  ctypes.byref(sm)), "fft_plan_schedule")
    return {"block": b.value, "wg_cap": c.value, "chunk_bytes": ch.value, "order": o.value, "small_side": sm.value}


def fft_plan_layout(plan):
    rb, w, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    ch = ctypes.c_int64()
    check(lib().fft_plan_layout(plan, ctypes.byref(rb), ctypes.byref(w), ctypes.byref(ch), ctypes.byref(g)),
          "fft_plan_layout")
    return {"rows_per_block": rb.value, "cols_per_tile": w.value, "chunk_images": ch.value, "grad_runs": g.value}


FFT_TREE_MAX_LOG2_PROCS = 6
FFT_TREE_MAX_LOG2 = 20
TREE_STATS_FIELDS = ("products", "busy_ticks", "wait_ticks", "sent_to", "send_level")
TREE_STATS_INT64 = len(TREE_STATS_FIELDS) * (1 << FFT_TREE_MAX_LOG2_PROCS) + 1  # + status


def fft_plan_tree(n, log2_procs, flags=0):
    h = _P()
    check(lib().fft_plan_tree(ctypes.byref(h), int(n), int(log2_procs), int(flags)), "fft_plan_tree")
    return h


def fft_tree_exec(plan, inp, out, workspace, stats, spin_limit, stream):
    check(lib().fft_tree_exec(plan, inp, out, workspace, stats, int(spin_limit), stream), "fft_tree_exec")


def tree_stats_dict(raw, nproc):
    """fft_tree_stats read back as int64 values -> dict of per-process lists."""
    P = 1 << FFT_TREE_MAX_LOG2_PROCS
    out = {f: [int(v) for v in raw[i * P:i * P + nproc]] for i, f in enumerate(TREE_STATS_FIELDS)}
    out["status"] = int(raw[len(TREE_STATS_FIELDS) * P])
    return out


def fft_plan_destroy(plan):
    check(lib().fft_plan_destroy(plan), "fft_plan_destroy")


def make_mask(kind="none", data_ptr=None, sigma_f=0.0, cutoff=0.0, order=0, b=0.0, c1=0.0, c2=0.0):
    kinds = {"none": FFT_MASK_NONE, "tensor": FFT_MASK_TENSOR_F32, "gaussian": FFT_MASK_GAUSSIAN,
             "butterworth": FFT_MASK_BUTTERWORTH, "disc": FFT_MASK_DISC}
    m = fft_mask()
    m.kind = kinds[kind] if isinstance(kind, str) else int(kind)
    m.data = data_ptr
    m.sigma_f = sigma_f
    m.cutoff = cutoff
    m.order = order
    m.b = b
    m.c1 = c1
    m.c2 = c2
    return m
