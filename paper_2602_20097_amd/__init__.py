"""MI355X-native quantization-aware interpolation (QAI) post-pass.

A from-scratch gfx950 implementation of the decompression post-pass of Jiao
et al., "Mitigating Artifacts in Pre-quantization Based Scientific Data
Compressors with Quantization-aware Interpolation" (arXiv 2602.20097),
Algorithm 4.  Every step runs in the HIP kernels of ``libqai.so``; this module
only marshals torch tensors (device memory, the current stream) into the C
ABI of ``include/qai.h``.

    import torch, paper_2602_20097_amd as qai
    out = qai.mitigate(x_dec_cuda_f32, eb)                 # Algorithm 4
    out, taps = qai.mitigate(x_dec, eb, taps=True)         # with intermediates
    y = qai.QAIFunction.apply(x_dec, eta_t, power_t, eb)    # differentiable
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import QAIError, QAI_STATUS_QRANGE  # noqa: F401

__all__ = ["mitigate", "workspace_bytes", "device_status", "backward", "QAIFunction", "fit_params",
           "BatchPlan", "mitigate_batched", "copy_probe", "profile", "stage_times", "QAIError", "lib", "autotune",
           "tuning_cache_save", "tuning_cache_load", "tuning_cache_clear", "tuning_cache_size", "quality", "mitigate_blocks", "upload_code", "decode",
           "mitigate_coded"]


def lib():
    return _lib.load()


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_field(t, name="field"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return _lib.dims3(t.shape)


def workspace_bytes(shape):
    return int(lib().qai_workspace_bytes(_lib.dims3(shape)))


def new_workspace(shape, device=None):
    """A 256-byte aligned uint8 device tensor large enough for ``shape``."""
    n = workspace_bytes(shape)
    if n == 0:
        raise QAIError(-2, f"invalid shape {tuple(shape)}")
    return torch.empty(n, dtype=torch.uint8, device=device or "cuda")


_TAP_TYPES = dict(q=torch.int32, b1=torch.uint8, sb=torch.int8, s=torch.int8, d1sq=torch.int32,
                  b2=torch.uint8, d2sq=torch.int32, w=torch.float32)


def mitigate(field, eb, eta=0.9, power=1.0, *, taps=False, out=None, workspace=None, stream=None):
    """Run the QAI post-pass on a decompressed float32 CUDA tensor.

    ``eb`` is the absolute error bound of the pre-quantization (Eq. 1).
    Returns ``out`` or, with ``taps=True``, ``(out, dict_of_intermediates)``
    (``q``, ``b1``, ``sb``, ``s``, ``d1sq``, ``b2``, ``d2sq``, ``w``).
    ``workspace`` (optional) is a uint8 device tensor of at least
    ``workspace_bytes(field.shape)`` bytes; afterwards it holds the distance
    words the adjoint (``backward``) needs.
    """
    L = lib()
    dims = _check_field(field)
    if out is None:
        out = torch.empty_like(field)
    else:
        _check_field(out, "out")
        if out.shape != field.shape:
            raise ValueError("out has the wrong shape")
    if workspace is None:
        workspace = new_workspace(field.shape, field.device)
    tp = None
    tap_t = {}
    if taps:
        tap_t = {k: torch.empty(field.shape, dtype=v, device=field.device) for k, v in _TAP_TYPES.items()}
        tp = _lib.Taps(**{k: v.data_ptr() for k, v in tap_t.items()})
    prm = _lib.Params(float(eta), float(power), 0)
    rc = L.qai_mitigate_ex(ctypes.c_void_p(field.data_ptr()), dims, ctypes.c_float(eb), ctypes.byref(prm),
                           ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                           ctypes.c_void_p(out.data_ptr()), ctypes.byref(tp) if tp is not None else None,
                           _stream_ptr(stream))
    _lib.check(rc)
    return (out, tap_t) if taps else out


def mitigate_simple(field, eb, out=None, stream=None):
    """The allocate-inside entry point ``qai_mitigate`` (default parameters)."""
    L = lib()
    dims = _check_field(field)
    if out is None:
        out = torch.empty_like(field)
    _lib.check(L.qai_mitigate(ctypes.c_void_p(field.data_ptr()), dims, ctypes.c_float(eb),
                              ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def device_status(workspace, stream=None):
    flags = ctypes.c_uint32(0)
    _lib.check(lib().qai_device_status(ctypes.c_void_p(workspace.data_ptr()), _stream_ptr(stream),
                                       ctypes.byref(flags)))
    return int(flags.value)


def backward(grad_out, workspace, shape, eb, eta=0.9, power=1.0, stream=None):
    """Adjoint of step E: returns a float32 CUDA tensor ``[dL/deta, dL/dpower]``
    for a workspace filled by ``mitigate(..., workspace=ws)`` on the same shape."""
    L = lib()
    _check_field(grad_out, "grad_out")
    g = torch.empty(2, dtype=torch.float32, device=grad_out.device)
    prm = _lib.Params(float(eta), float(power), 0)
    _lib.check(L.qai_backward(ctypes.c_void_p(grad_out.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
                              workspace.numel(), _lib.dims3(shape), ctypes.c_float(eb), ctypes.byref(prm),
                              ctypes.c_void_p(g.data_ptr()), _stream_ptr(stream)))
    return g


class QAIFunction(torch.autograd.Function):
    """Differentiable QAI (project addition): ``y = QAIFunction.apply(x_dec,
    eta, power, eb)`` with ``eta`` and ``power`` 0-dim float32 tensors.  The
    distance transforms are held fixed; gradients flow to the decompressed
    values (identity) and to ``eta`` and ``power``."""

    @staticmethod
    def forward(ctx, x_dec, eta, power, eb):
        ws = new_workspace(x_dec.shape, x_dec.device)
        e, p = float(eta), float(power)
        out = mitigate(x_dec.detach().contiguous(), eb, e, p, workspace=ws)
        ctx.save_for_backward(ws)
        ctx.meta = (tuple(x_dec.shape), float(eb), e, p, eta.dtype, power.dtype)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        (ws,) = ctx.saved_tensors
        shape, eb, e, p, edt, pdt = ctx.meta
        g = backward(grad_out.contiguous().float(), ws, shape, eb, e, p)
        return grad_out, g[0].to(edt), g[1].to(pdt), None


def fit_params(x_dec, x_orig, eb, steps=50, eta0=0.9, power0=1.0, fit_power=True, history=10):
    """Fit eta (and optionally the IDW power) for one field by minimising the
    MSE between the compensated and the original data: ``steps`` L-BFGS
    iterations with a strong-Wolfe line search (the MSE taken relative to its
    starting value), on float64 parameters (the
    power as exp(theta), so that every trial value stays positive), each loss
    evaluation one forward pass and one adjoint on the GPU.  Returns
    ``(eta, power, history_of_mse)`` (the MSE after each iteration)."""
    dev = x_dec.device
    eta = torch.tensor(float(eta0), dtype=torch.float64, device=dev, requires_grad=True)
    theta = torch.tensor(float(np.log(power0)), dtype=torch.float64, device=dev, requires_grad=fit_power)
    params = [eta, theta] if fit_power else [eta]
    # one iteration per step, with up to 25 loss evaluations for its line search
    opt = torch.optim.LBFGS(params, lr=1.0, max_iter=1, max_eval=25, history_size=history,
                            line_search_fn="strong_wolfe")
    xo = x_orig.double()

    def loss_fn():
        pw = torch.exp(theta)
        y = QAIFunction.apply(x_dec, eta, pw, eb)
        return torch.mean((y.double() - xo) ** 2)

    with torch.no_grad():
        scale = 1.0 / max(float(loss_fn()), 1e-300)  # the optimiser sees the MSE relative to its start

    def closure():
        opt.zero_grad()
        loss = loss_fn() * scale
        loss.backward()
        return loss

    hist = []
    for _ in range(steps):
        opt.step(closure)
        with torch.no_grad():
            hist.append(float(loss_fn()))
    return float(eta.detach()), float(torch.exp(theta).detach()), hist


class BatchPlan:
    """Batched form: many float32 CUDA fields of uneven shapes run by one
    hipGraph launch (``qai_batch_plan_*``).  ``outs`` and the workspace are
    allocated here unless given; the plan keeps references to every tensor it
    uses.  ``autotune=True`` takes the autotuner's setting for each distinct
    shape (timed on its first field unless cached); ``tune_each=True`` also
    times the pass-algorithm variants on every field (results are unchanged by
    either)."""

    def __init__(self, fields, ebs, outs=None, eta=0.9, power=1.0, autotune=True, workspace=None, stream=None,
                 tune_each=False):
        L = lib()
        if len(fields) != len(ebs) or not fields:
            raise ValueError("one error bound per field, at least one field")
        self.fields = list(fields)
        for f in self.fields:
            _check_field(f)
        self.outs = list(outs) if outs is not None else [torch.empty_like(f) for f in self.fields]
        n = len(self.fields)
        dims = (_lib.Dims * n)(*[_lib.dims3(f.shape) for f in self.fields])
        need = int(L.qai_batch_workspace_bytes(n, dims))
        if need == 0:
            raise QAIError(-2, "invalid field shapes")
        dev = self.fields[0].device
        self.workspace = workspace if workspace is not None else torch.empty(need, dtype=torch.uint8, device=dev)
        fp = (ctypes.c_void_p * n)(*[f.data_ptr() for f in self.fields])
        op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in self.outs])
        eb = (ctypes.c_float * n)(*[float(e) for e in ebs])
        prm = _lib.Params(float(eta), float(power), 0)
        h = ctypes.c_void_p()
        _lib.check(L.qai_batch_plan_create(n, fp, dims, eb, op, ctypes.byref(prm),
                                           (_lib.QAI_BATCH_AUTOTUNE | (_lib.QAI_BATCH_TUNE_EACH if tune_each else 0))
                                           if autotune else 0,
                                           ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                           _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self.n = n

    def launch(self, stream=None):
        """Replay the graph: every output is (re)written."""
        _lib.check(lib().qai_batch_plan_launch(self._h, _stream_ptr(stream)))
        return self.outs

    def launch_per_field(self, stream=None):
        """The same batch as separate launches, field after field."""
        _lib.check(lib().qai_batch_plan_launch_per_field(self._h, _stream_ptr(stream)))
        return self.outs

    def tuning(self, i):
        t = _lib.Tuning()
        _lib.check(lib().qai_batch_plan_tuning(self._h, int(i), ctypes.byref(t)))
        return {k: (list(getattr(t, k)) if hasattr(getattr(t, k), "__len__") else int(getattr(t, k)))
                for k in TUNING_FIELDS}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().qai_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mitigate_batched(fields, ebs, eta=0.9, power=1.0, autotune=False, stream=None):
    """Run the post-pass on a list of fields with one graph launch; returns
    the list of outputs."""
    plan = BatchPlan(fields, ebs, eta=eta, power=power, autotune=autotune, stream=stream)
    outs = plan.launch(stream)
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    plan.close()
    return outs


def copy_probe(src, dst, stream=None):
    """Device copy of ``src`` into ``dst`` (same number of bytes, multiple of 4)."""
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n or n % 4:
        raise ValueError("copy_probe needs equal sizes that are multiples of 4 bytes")
    _lib.check(lib().qai_copy_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), n // 4,
                                    _stream_ptr(stream)))


TUNING_FIELDS = ("edt1_algo", "edt2_algo", "edt1_ring", "edt2_ring", "tile_log2", "seed_rows", "seed_planes",
                 "window_threads", "force_wide")


def get_tuning():
    """The current launch setting as a dict (see qai_tuning in include/qai.h)."""
    t = _lib.Tuning()
    _lib.check(lib().qai_tuning_get(ctypes.byref(t)))
    out = {}
    for k in TUNING_FIELDS:
        v = getattr(t, k)
        out[k] = list(v) if hasattr(v, "__len__") else int(v)
    return out


def set_tuning(cfg=None, **kw):
    """Replace the launch setting; ``None`` restores the defaults.  Keys not
    given keep their current values."""
    if cfg is None and not kw:
        _lib.check(lib().qai_tuning_set(None))
        return get_tuning()
    cur = get_tuning()
    cur.update(cfg or {})
    cur.update(kw)
    t = _lib.Tuning()
    for k in TUNING_FIELDS:
        v = cur[k]
        if isinstance(v, (list, tuple)):
            getattr(t, k)[:] = [int(x) for x in v]
        else:
            setattr(t, k, int(v))
    _lib.check(lib().qai_tuning_set(ctypes.byref(t)))
    return get_tuning()


def autotune(field, eb, stream=None):
    """Time the candidate launch settings on ``field`` and cache the fastest
    for its shape (used by later calls while the process-wide setting is the
    default); returns the chosen setting as a dict."""
    L = lib()
    dims = _check_field(field)
    ws = new_workspace(field.shape, field.device)
    out = torch.empty_like(field)
    t = _lib.Tuning()
    _lib.check(L.qai_autotune(ctypes.c_void_p(field.data_ptr()), dims, ctypes.c_float(eb),
                              ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(out.data_ptr()),
                              _stream_ptr(stream), ctypes.byref(t)))
    return {k: (list(getattr(t, k)) if hasattr(getattr(t, k), "__len__") else int(getattr(t, k)))
            for k in TUNING_FIELDS}


def tuning_cache_save(path):
    _lib.check(lib().qai_tuning_cache_save(str(path).encode()))


def tuning_cache_load(path):
    _lib.check(lib().qai_tuning_cache_load(str(path).encode()))


def tuning_cache_clear():
    _lib.check(lib().qai_tuning_cache_clear())


def tuning_cache_size():
    return int(lib().qai_tuning_cache_size())


def mitigate_blocks(field, eb, blocks=(2, 2, 2), mode="approximate", eta=0.9, power=1.0, out=None, stream=None):
    """The post-pass with the field cut into a grid of blocks (the paper's
    distributed strategies, Section VI-B): ``mode`` "ep" (each block alone) or
    "approximate" (one-layer exchanges of the data and of the propagated
    signs, local EDTs).  The exact strategy is ``mitigate`` itself."""
    L = lib()
    dims = _check_field(field)
    if mode not in _lib.BLOCK_MODES:
        raise ValueError(f"mode must be one of {sorted(_lib.BLOCK_MODES)}")
    m = _lib.BLOCK_MODES[mode]
    blk = (ctypes.c_int32 * 3)(*[int(b) for b in ((1,) * (3 - len(blocks)) + tuple(blocks))])
    nb = int(L.qai_blocks_workspace_bytes(dims, blk, m))
    if nb == 0:
        raise QAIError(-1, f"invalid blocks {tuple(blocks)} for shape {tuple(field.shape)}")
    ws = torch.empty(nb, dtype=torch.uint8, device=field.device)
    if out is None:
        out = torch.empty_like(field)
    prm = _lib.Params(float(eta), float(power), 0)
    _lib.check(L.qai_mitigate_blocks(ctypes.c_void_p(field.data_ptr()), dims, ctypes.c_float(eb), ctypes.byref(prm),
                                     blk, m, ctypes.c_void_p(ws.data_ptr()), nb, ctypes.c_void_p(out.data_ptr()),
                                     _stream_ptr(stream)))
    return out


def upload_code(code, device="cuda"):
    """Device copies of a segment code (the dict of ``synth.encode_indices``):
    returns a dict of int32 / int64 / int32 tensors plus its shape."""
    import numpy as _np
    return {"base": torch.from_numpy(_np.ascontiguousarray(code["base"])).to(device),
            "meta": torch.from_numpy(_np.ascontiguousarray(code["meta"]).view(_np.int64)).to(device),
            "payload": torch.from_numpy(_np.ascontiguousarray(code["payload"]).view(_np.int32)).to(device),
            "seg_len": int(code["seg_len"]), "shape": tuple(code["shape"])}


def _coded(dcode):
    return _lib.Coded(dcode["base"].data_ptr(), dcode["meta"].data_ptr(), dcode["payload"].data_ptr(),
                      dcode["payload"].numel(), dcode["seg_len"])


def decode(dcode, eb, out=None, stream=None):
    """x' = 2 eb q from a device segment code (``upload_code``)."""
    shape = dcode["shape"]
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=dcode["base"].device)
    c = _coded(dcode)
    _lib.check(lib().qai_decode(ctypes.byref(c), _lib.dims3(shape), ctypes.c_float(eb),
                                ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def mitigate_coded(dcode, eb, eta=0.9, power=1.0, out=None, workspace=None, stream=None):
    """The post-pass from a device segment code (``upload_code``): the first
    seed pass decodes the indices and writes x' into ``out``, which the later
    stages read in place; returns ``out``."""
    L = lib()
    shape = dcode["shape"]
    dev = dcode["base"].device
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=dev)
    if workspace is None:
        workspace = new_workspace(shape, dev)
    c = _coded(dcode)
    prm = _lib.Params(float(eta), float(power), 0)
    _lib.check(L.qai_mitigate_coded(ctypes.byref(c), _lib.dims3(shape), ctypes.c_float(eb), ctypes.byref(prm),
                                    ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                    ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def quality(orig, dec, stream=None, sync=True):
    """SSIM (Eq. 3, 7-voxel windows at stride 2) and PSNR (Eq. 4) of ``dec``
    against ``orig`` on the GPU.  Returns a dict ``{"ssim", "psnr", "mse",
    "range"}`` (``sync=True``) or the device float64 tensor of those four."""
    L = lib()
    dims = _check_field(orig, "orig")
    _check_field(dec, "dec")
    if dec.shape != orig.shape:
        raise ValueError("orig and dec differ in shape")
    nb = int(L.qai_quality_workspace_bytes(dims))
    if nb == 0:
        raise QAIError(-2, f"invalid shape {tuple(orig.shape)}")
    ws = torch.empty(nb, dtype=torch.uint8, device=orig.device)
    res = torch.empty(4, dtype=torch.float64, device=orig.device)
    _lib.check(L.qai_quality(ctypes.c_void_p(orig.data_ptr()), ctypes.c_void_p(dec.data_ptr()), dims,
                             ctypes.c_void_p(ws.data_ptr()), nb, ctypes.c_void_p(res.data_ptr()),
                             _stream_ptr(stream)))
    if not sync:
        return res
    v = res.cpu().tolist()
    return {"ssim": v[0], "psnr": v[1], "mse": v[2], "range": v[3]}


def profile(on=True):
    _lib.check(lib().qai_profile_enable(1 if on else 0))


def stage_times(reset=True):
    """Milliseconds per stage accumulated since the last reset (synchronises)."""
    L = lib()
    ms = (ctypes.c_double * 32)()
    names = (ctypes.c_char_p * 32)()
    k = ctypes.c_int(0)
    _lib.check(L.qai_stage_times(ms, names, 32, ctypes.byref(k), 1 if reset else 0))
    return {names[i].decode(): ms[i] for i in range(min(k.value, 32))}
