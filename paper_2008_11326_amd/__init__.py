"""MI355X-native GPP self-energy reduction (paper Sec. II-A) behind a C ABI.

The computation runs in hand-written HIP kernels for gfx950 (libgpp.so,
include/gpp.h).  This module only marshals torch CUDA tensors (device
memory and the current stream) into that ABI.

    ach, asx = sigma_fwd(aqsmtemp, aqsntemp, I_eps_array, wtilde_array,
                         vcoul, wx_array, nvband)
    ach, asx, qp = sigma_qp(..., nvband, freq_step, energy, vxc)  # + Sigma(E), dSigma/dE, Z, E_qp
    grads = sigma_bwd(..., grad_achtemp, grad_asxtemp)   # adjoint
    ach, asx = sigma(...)            # differentiable (GppSigma autograd.Function)
    plan = Plan([dims_0, dims_1, ...])          # many states, one launch
    ach, asx = sigma_batched(plan, [state_0_tensors, state_1_tensors, ...])

Layouts (row-major, last index fastest): aqsmtemp/aqsntemp complex128
[number_bands, ncouls]; I_eps_array/wtilde_array complex128 [ngpown, ncouls];
vcoul float64 [ncouls]; wx_array float64 [nfreq, number_bands].  Outputs
are complex128 [nfreq].
"""
from __future__ import annotations

import ctypes as C

from . import _lib
from ._lib import GppError, MAX_NFREQ

__all__ = ["sigma_fwd", "sigma_fwd_noalloc", "sigma_qp", "sigma_bwd", "sigma", "GppSigma", "Plan", "sigma_batched",
           "fwd_workspace_bytes", "bwd_workspace_bytes", "GppError", "MAX_NFREQ",
           "library_path"]


def library_path() -> str:
    return _lib.LIB_PATH


def _torch():
    import torch
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t.numel() > 0 else C.c_void_p(0)


def _check_tensor(name, t, dtype, shape, device):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.is_conj() or t.is_neg():
        # a lazy conjugate/negative view: its memory holds the unconjugated
        # values, which the kernels would read as they are
        raise ValueError(f"{name} is a lazy conjugate or negative view; pass "
                         f"{name}.resolve_conj().resolve_neg()")


def _prepare(aqsmtemp, aqsntemp, I_eps_array, wtilde_array, vcoul, wx_array,
             nvband):
    torch = _torch()
    if aqsntemp.dim() != 2 or I_eps_array.dim() != 2 or wx_array.dim() != 2:
        raise ValueError("aqsntemp, I_eps_array and wx_array must be 2-D")
    nb, ng = aqsntemp.shape
    npw = I_eps_array.shape[0]
    nw = wx_array.shape[0]
    dev = aqsntemp.device
    if dev.type != "cuda":
        raise ValueError("inputs must be CUDA (HIP) tensors")
    c128, f64 = torch.complex128, torch.float64
    _check_tensor("aqsmtemp", aqsmtemp, c128, (nb, ng), dev)
    _check_tensor("aqsntemp", aqsntemp, c128, (nb, ng), dev)
    _check_tensor("I_eps_array", I_eps_array, c128, (npw, ng), dev)
    _check_tensor("wtilde_array", wtilde_array, c128, (npw, ng), dev)
    _check_tensor("vcoul", vcoul, f64, (ng,), dev)
    _check_tensor("wx_array", wx_array, f64, (nw, nb), dev)
    dims = _lib.dims_struct(nb, nvband, ng, npw, nw)
    ins = _lib.GppInputs(_ptr(aqsmtemp), _ptr(aqsntemp), _ptr(I_eps_array),
                         _ptr(wtilde_array), _ptr(vcoul), _ptr(wx_array))
    return dims, ins, dev


def fwd_workspace_bytes(number_bands, nvband, ncouls, ngpown, nfreq) -> int:
    d = _lib.dims_struct(number_bands, nvband, ncouls, ngpown, nfreq)
    return int(_lib.load().gpp_sigma_fwd_workspace(C.byref(d)))


def sigma_fwd(aqsmtemp, aqsntemp, I_eps_array, wtilde_array, vcoul, wx_array,
              nvband: int, *, out=None, workspace=None, stream=None):
    """achtemp, asxtemp (complex128 [nfreq] each) via gpp_sigma_fwd.

    `out` may be a pair of preallocated complex128 [nfreq] tensors and
    `workspace` a uint8 tensor of at least fwd_workspace_bytes(...) bytes;
    `stream` defaults to torch's current stream on the inputs' device."""
    torch = _torch()
    lib = _lib.load()
    dims, ins, dev = _prepare(aqsmtemp, aqsntemp, I_eps_array, wtilde_array,
                              vcoul, wx_array, nvband)
    nw = dims.nfreq
    if out is None:
        ach = torch.empty(nw, dtype=torch.complex128, device=dev)
        asx = torch.empty(nw, dtype=torch.complex128, device=dev)
    else:
        ach, asx = out
        _check_tensor("achtemp", ach, torch.complex128, (nw,), dev)
        _check_tensor("asxtemp", asx, torch.complex128, (nw,), dev)
    need = int(lib.gpp_sigma_fwd_workspace(C.byref(dims)))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    with torch.cuda.device(dev):
        st = lib.gpp_sigma_fwd(C.byref(dims), C.byref(ins), _ptr(ach), _ptr(asx),
                               _ptr(workspace), workspace.numel(),
                               C.c_void_p(stream))
    _lib.check(st, "gpp_sigma_fwd")
    return ach, asx


def sigma_fwd_noalloc(aqsmtemp, aqsntemp, I_eps_array, wtilde_array, vcoul, wx_array,
                      nvband: int, *, out, stream=None):
    """sigma_fwd through gpp_sigma_fwd_noalloc, which allocates nothing: its
    workspace is a fixed array inside the library (include/gpp.h).  `out`
    must be a pair of preallocated complex128 [nfreq] tensors."""
    torch = _torch()
    lib = _lib.load()
    dims, ins, dev = _prepare(aqsmtemp, aqsntemp, I_eps_array, wtilde_array,
                              vcoul, wx_array, nvband)
    ach, asx = out
    _check_tensor("achtemp", ach, torch.complex128, (dims.nfreq,), dev)
    _check_tensor("asxtemp", asx, torch.complex128, (dims.nfreq,), dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    with torch.cuda.device(dev):
        st = lib.gpp_sigma_fwd_noalloc(C.byref(dims), C.byref(ins), _ptr(ach), _ptr(asx),
                                       C.c_void_p(stream))
    _lib.check(st, "gpp_sigma_fwd_noalloc")
    return ach, asx


def sigma_qp(aqsmtemp, aqsntemp, I_eps_array, wtilde_array, vcoul, wx_array,
             nvband: int, freq_step: float, energy: float = 0.0, vxc: float = 0.0, *,
             out=None, workspace=None, stream=None):
    """achtemp, asxtemp and the quasiparticle quantities via gpp_sigma_qp:
    returns (achtemp, asxtemp, qp) with qp a float64 [6] tensor holding
    Sigma(E) re/im, dSigma/dE re/im, Z and E_qp (include/gpp.h).  The nfreq
    (odd) frequencies are energy + (w - (nfreq-1)/2) freq_step."""
    torch = _torch()
    lib = _lib.load()
    dims, ins, dev = _prepare(aqsmtemp, aqsntemp, I_eps_array, wtilde_array,
                              vcoul, wx_array, nvband)
    nw = dims.nfreq
    if out is None:
        ach = torch.empty(nw, dtype=torch.complex128, device=dev)
        asx = torch.empty(nw, dtype=torch.complex128, device=dev)
        qp = torch.empty(6, dtype=torch.float64, device=dev)
    else:
        ach, asx, qp = out
        _check_tensor("achtemp", ach, torch.complex128, (nw,), dev)
        _check_tensor("asxtemp", asx, torch.complex128, (nw,), dev)
        _check_tensor("qp", qp, torch.float64, (6,), dev)
    need = int(lib.gpp_sigma_fwd_workspace(C.byref(dims)))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    with torch.cuda.device(dev):
        st = lib.gpp_sigma_qp(C.byref(dims), C.byref(ins), float(freq_step), float(energy),
                              float(vxc), _ptr(ach), _ptr(asx), _ptr(qp), _ptr(workspace),
                              workspace.numel(), C.c_void_p(stream))
    _lib.check(st, "gpp_sigma_qp")
    return ach, asx, qp


def bwd_workspace_bytes(number_bands, nvband, ncouls, ngpown, nfreq) -> int:
    d = _lib.dims_struct(number_bands, nvband, ncouls, ngpown, nfreq)
    return int(_lib.load().gpp_sigma_bwd_workspace(C.byref(d)))


def sigma_bwd(aqsmtemp, aqsntemp, I_eps_array, wtilde_array, vcoul, wx_array,
              nvband: int, grad_achtemp, grad_asxtemp, *,
              want=(True, True, True, True), workspace=None, stream=None):
    """Vector-Jacobian product of sigma_fwd via gpp_sigma_bwd.

    Returns (grad_aqsmtemp, grad_aqsntemp, grad_I_eps_array,
    grad_wtilde_array), each a complex128 tensor shaped like its input or
    None where `want` is False.  Gradients follow PyTorch's convention
    dL/dRe z + i dL/dIm z for L = sum Re(conj(g) * output)."""
    torch = _torch()
    lib = _lib.load()
    dims, ins, dev = _prepare(aqsmtemp, aqsntemp, I_eps_array, wtilde_array,
                              vcoul, wx_array, nvband)
    nw = dims.nfreq
    _check_tensor("grad_achtemp", grad_achtemp, torch.complex128, (nw,), dev)
    _check_tensor("grad_asxtemp", grad_asxtemp, torch.complex128, (nw,), dev)
    shapes = (aqsmtemp.shape, aqsntemp.shape, I_eps_array.shape, wtilde_array.shape)
    outs = [torch.empty(sh, dtype=torch.complex128, device=dev) if w else None
            for sh, w in zip(shapes, want)]
    need = int(lib.gpp_sigma_bwd_workspace(C.byref(dims)))
    if workspace is None:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    p = lambda t: _ptr(t) if t is not None else C.c_void_p(0)
    with torch.cuda.device(dev):
        st = lib.gpp_sigma_bwd(C.byref(dims), C.byref(ins), _ptr(grad_achtemp),
                               _ptr(grad_asxtemp), p(outs[0]), p(outs[1]), p(outs[2]),
                               p(outs[3]), _ptr(workspace), workspace.numel(),
                               C.c_void_p(stream))
    _lib.check(st, "gpp_sigma_bwd")
    return tuple(outs)


def _make_function():
    torch = _torch()

    class GppSigma(torch.autograd.Function):
        """(achtemp, asxtemp) = GPP reduction; backward runs the hand-written
        adjoint kernels (gpp_sigma_bwd).  vcoul, wx_array and nvband get no
        gradient."""

        @staticmethod
        def forward(ctx, aqsmtemp, aqsntemp, I_eps_array, wtilde_array, vcoul,
                    wx_array, nvband):
            ach, asx = sigma_fwd(aqsmtemp, aqsntemp, I_eps_array, wtilde_array,
                                 vcoul, wx_array, nvband)
            ctx.save_for_backward(aqsmtemp, aqsntemp, I_eps_array, wtilde_array,
                                  vcoul, wx_array)
            ctx.nvband = int(nvband)
            return ach, asx

        @staticmethod
        def backward(ctx, g_ach, g_asx):
            ins = ctx.saved_tensors
            nw = ins[5].shape[0]
            dev = ins[0].device
            zero = lambda: torch.zeros(nw, dtype=torch.complex128, device=dev)
            fix = lambda g: g.resolve_conj().resolve_neg().contiguous()
            g_ach = zero() if g_ach is None else fix(g_ach)
            g_asx = zero() if g_asx is None else fix(g_asx)
            want = tuple(bool(x) for x in ctx.needs_input_grad[:4])
            if not any(want):
                return (None,) * 7
            grads = sigma_bwd(*ins, ctx.nvband, g_ach, g_asx, want=want)
            return grads + (None, None, None)

    return GppSigma


_fn = None


def __getattr__(name):
    # GppSigma is built on first use so importing the package needs no torch
    global _fn
    if name == "GppSigma":
        if _fn is None:
            _fn = _make_function()
        return _fn
    raise AttributeError(name)


def sigma(aqsmtemp, aqsntemp, I_eps_array, wtilde_array, vcoul, wx_array, nvband):
    """Differentiable (achtemp, asxtemp) through GppSigma."""
    return __getattr__("GppSigma").apply(aqsmtemp, aqsntemp, I_eps_array,
                                         wtilde_array, vcoul, wx_array, nvband)


class Plan:
    """Batched-forward plan (gpp_plan_create): the states' sizes as
    (number_bands, nvband, ncouls, ngpown, nfreq) tuples.  Create it with
    the target device current; release with close() (or let it be
    collected)."""

    def __init__(self, dims):
        lib = _lib.load()
        self.dims = [tuple(int(v) for v in d) for d in dims]
        arr = (_lib.GppDims * len(self.dims))(*[_lib.GppDims(*d) for d in self.dims])
        handle = C.c_void_p()
        _lib.check(lib.gpp_plan_create(len(self.dims), arr, C.byref(handle)),
                   "gpp_plan_create")
        self._h = handle
        self.workspace_bytes = int(lib.gpp_plan_workspace(handle))

    def info(self) -> dict:
        inf = _lib.GppPlanInfo()
        _lib.check(_lib.load().gpp_plan_get_info(self._h, C.byref(inf)),
                   "gpp_plan_get_info")
        return {f: getattr(inf, f) for f, _ in inf._fields_}

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().gpp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_STATE_KEYS = ("aqsmtemp", "aqsntemp", "I_eps_array", "wtilde_array", "vcoul",
               "wx_array")


def sigma_batched(plan: Plan, states, *, out=None, workspace=None, stream=None):
    """achtemp, asxtemp (complex128 [nstates, nfreq]) for every state via
    gpp_sigma_batched.  `states` is a sequence of dicts (or 6-tuples) of
    CUDA tensors in sigma_fwd's layouts, matching the plan's sizes."""
    torch = _torch()
    lib = _lib.load()
    if len(states) != len(plan.dims):
        raise ValueError(f"plan has {len(plan.dims)} states, got {len(states)}")
    ins = (_lib.GppInputs * len(states))()
    dev = None
    for k, (st, d) in enumerate(zip(states, plan.dims)):
        if not isinstance(st, dict):
            st = dict(zip(_STATE_KEYS, st))
        dims, one, dv = _prepare(*[st[key] for key in _STATE_KEYS], d[1])
        if (dims.number_bands, dims.nvband, dims.ncouls, dims.ngpown, dims.nfreq) != d:
            got = (dims.number_bands, dims.nvband, dims.ncouls, dims.ngpown, dims.nfreq)
            raise ValueError(f"state {k}: tensors have sizes {got}, plan expects {d}")
        if dev is not None and dv != dev:
            raise ValueError("all states must be on one device")
        dev = dv
        ins[k] = one
    nw = plan.dims[0][4]
    shape = (len(states), nw)
    if out is None:
        ach = torch.empty(shape, dtype=torch.complex128, device=dev)
        asx = torch.empty(shape, dtype=torch.complex128, device=dev)
    else:
        ach, asx = out
        _check_tensor("achtemp", ach, torch.complex128, shape, dev)
        _check_tensor("asxtemp", asx, torch.complex128, shape, dev)
    if workspace is None:
        workspace = torch.empty(max(plan.workspace_bytes, 256), dtype=torch.uint8,
                                device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    with torch.cuda.device(dev):
        st = lib.gpp_sigma_batched(plan._h, ins, _ptr(ach), _ptr(asx), _ptr(workspace),
                                   workspace.numel(), C.c_void_p(stream))
    _lib.check(st, "gpp_sigma_batched")
    return ach, asx
