"""ctypes binding of the learned-warm-start kernels (C ABI in
``include/lbm_nn.h``), argument marshalling only.  Tensors are torch
tensors on the GPU: bf16 activations/weights as ``torch.bfloat16`` (passed
as raw bit patterns), everything else float32/float64/uint8."""
from __future__ import annotations

import ctypes

from . import lbm

NN_EXPORTED = ["nn_conv3d_fwd", "nn_conv3d_fwd_upcat", "nn_conv3d_dgrad", "nn_conv3d_wgrad", "nn_conv3d_wgrad_workspace",
               "nn_lrelu_bwd", "nn_up_concat", "nn_split_down", "nn_masked_mse",
               "nn_masked_mse_noalloc", "nn_adam_step", "nn_prepare_input", "nn_prepare_input_dist",
               "nn_velocity_labels", "nn_velocity_out",
               "nn_to_bf16"]


class ConvDesc(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("d", ctypes.c_int32), ("h", ctypes.c_int32),
                ("w", ctypes.c_int32), ("c_in", ctypes.c_int32), ("c_out", ctypes.c_int32),
                ("c_store", ctypes.c_int32), ("stride", ctypes.c_int32), ("taps", ctypes.c_int32),
                ("act", ctypes.c_int32), ("slope", ctypes.c_float), ("out_f32", ctypes.c_int32)]


_ready = False


def _lib():
    global _ready
    lib = lbm.load()
    if not _ready:
        vp = ctypes.c_void_p
        D = ctypes.POINTER(ConvDesc)
        i64 = ctypes.c_int64
        i32 = ctypes.c_int32
        f32 = ctypes.c_float
        f64 = ctypes.c_double
        sig = {
            "nn_conv3d_fwd": [D, vp, vp, vp, vp, vp],
            "nn_conv3d_fwd_upcat": [D, vp, i32, vp, vp, vp, vp, vp],
            "nn_conv3d_dgrad": [D, vp, vp, vp, vp, i32, vp],
            "nn_conv3d_wgrad": [D, vp, vp, vp, vp, vp, vp],
            "nn_conv3d_wgrad_workspace": [D],
            "nn_lrelu_bwd": [vp, vp, vp, i64, f32, vp],
            "nn_up_concat": [vp, vp, vp, i32, i32, i32, i32, i32, i32, vp],
            "nn_split_down": [vp, vp, vp, i32, i32, i32, i32, i32, i32, vp],
            "nn_masked_mse": [vp, vp, vp, i64, vp, vp, vp, vp],
            "nn_masked_mse_noalloc": [vp, vp, vp, i64, vp, vp, vp],
            "nn_adam_step": [vp, vp, vp, vp, vp, i64, f64, f64, f64, f64, i32, vp],
            "nn_prepare_input": [vp, vp, i64, i32, vp],
            "nn_prepare_input_dist": [vp, vp, i32, i32, i32, f32, vp, vp],
            "nn_velocity_labels": [vp, vp, ctypes.c_double, vp, i64, vp],
            "nn_velocity_out": [vp, vp, ctypes.c_double, vp, i64, vp],
            "nn_to_bf16": [vp, vp, i64, vp],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int64 if name == "nn_conv3d_wgrad_workspace" else ctypes.c_int
        _ready = True
    return lib


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s(stream):
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(st.cuda_stream)


def _check(rc, where):
    if rc != 0:
        raise RuntimeError("%s failed (%d): %s" % (where, rc, lbm.load().lbm_last_error().decode()))


def desc(batch, d, h, w, c_in, c_out, c_store=None, stride=1, taps=27, act=True, slope=0.1,
         out_f32=False) -> ConvDesc:
    x = ConvDesc()
    x.batch, x.d, x.h, x.w = batch, d, h, w
    x.c_in, x.c_out = c_in, c_out
    x.c_store = c_out if c_store is None else c_store
    x.stride, x.taps, x.act, x.slope, x.out_f32 = stride, taps, int(act), slope, int(out_f32)
    return x


def conv_fwd(dsc, x, w, bias, y, stream=None):
    _check(_lib().nn_conv3d_fwd(ctypes.byref(dsc), _p(x), _p(w), _p(bias), _p(y), _s(stream)),
           "nn_conv3d_fwd")


def conv_fwd_upcat(dsc, coarse, c_coarse, skip, w, bias, y, stream=None):
    """conv_fwd of up_concat(coarse, skip) without forming the concatenation."""
    _check(_lib().nn_conv3d_fwd_upcat(ctypes.byref(dsc), _p(coarse), int(c_coarse), _p(skip), _p(w),
                                      _p(bias), _p(y), _s(stream)), "nn_conv3d_fwd_upcat")


def conv_dgrad(dsc, dy, w, w_t, dx, accumulate=False, stream=None):
    _check(_lib().nn_conv3d_dgrad(ctypes.byref(dsc), _p(dy), _p(w), _p(w_t), _p(dx),
                                  int(accumulate), _s(stream)), "nn_conv3d_dgrad")


def wgrad_workspace(dsc) -> int:
    n = _lib().nn_conv3d_wgrad_workspace(ctypes.byref(dsc))
    if n < 0:
        raise RuntimeError("bad descriptor: " + lbm.load().lbm_last_error().decode())
    return int(n)


def conv_wgrad(dsc, x, dy, dw, db, workspace, stream=None):
    _check(_lib().nn_conv3d_wgrad(ctypes.byref(dsc), _p(x), _p(dy), _p(dw), _p(db), _p(workspace),
                                  _s(stream)), "nn_conv3d_wgrad")


def lrelu_bwd(dx, y, dy_pre, slope, stream=None):
    _check(_lib().nn_lrelu_bwd(_p(dx), _p(y), _p(dy_pre), dx.numel(), slope, _s(stream)),
           "nn_lrelu_bwd")


def up_concat(coarse, skip, cat, batch, d, h, w, c1, c2, stream=None):
    _check(_lib().nn_up_concat(_p(coarse), _p(skip), _p(cat), batch, d, h, w, c1, c2, _s(stream)),
           "nn_up_concat")


def split_down(dcat, dcoarse, dskip, batch, d, h, w, c1, c2, stream=None):
    _check(_lib().nn_split_down(_p(dcat), _p(dcoarse), _p(dskip), batch, d, h, w, c1, c2,
                                _s(stream)), "nn_split_down")


def masked_mse(pred, target, mask, dy, loss, workspace, stream=None):
    _check(_lib().nn_masked_mse(_p(pred), _p(target), _p(mask), mask.numel(), _p(dy), _p(loss),
                                _p(workspace), _s(stream)), "nn_masked_mse")


def masked_mse_noalloc(pred, target, mask, dy, loss, stream=None, n=None):
    """nn_masked_mse on the library's own device scratch (no workspace).
    ``n``: voxel count (default: mask.numel())."""
    _check(_lib().nn_masked_mse_noalloc(_p(pred), _p(target), _p(mask),
                                        mask.numel() if n is None else int(n), _p(dy), _p(loss),
                                        _s(stream)), "nn_masked_mse_noalloc")


def adam_step(param, grad, m, v, param_bf16, lr, beta1, beta2, eps, t, stream=None):
    _check(_lib().nn_adam_step(_p(param), _p(grad), _p(m), _p(v), _p(param_bf16), param.numel(),
                               lr, beta1, beta2, eps, int(t), _s(stream)), "nn_adam_step")


def prepare_input(mask, x, c_pad, stream=None):
    _check(_lib().nn_prepare_input(_p(mask), _p(x), mask.numel(), c_pad, _s(stream)),
           "nn_prepare_input")


def prepare_input_dist(mask, x, batch, n, c_pad, dmax, work, stream=None):
    _check(_lib().nn_prepare_input_dist(_p(mask), _p(x), int(batch), int(n), int(c_pad),
                                        float(dmax), _p(work), _s(stream)),
           "nn_prepare_input_dist")


def velocity_labels(u, mask, scale, out, stream=None):
    _check(_lib().nn_velocity_labels(_p(u), _p(mask), float(scale), _p(out), mask.numel(),
                                     _s(stream)), "nn_velocity_labels")


def velocity_out(pred, mask, scale, u, stream=None):
    _check(_lib().nn_velocity_out(_p(pred), _p(mask), float(scale), _p(u), mask.numel(),
                                  _s(stream)), "nn_velocity_out")


def to_bf16(src, dst, stream=None):
    _check(_lib().nn_to_bf16(_p(src), _p(dst), src.numel(), _s(stream)), "nn_to_bf16")
