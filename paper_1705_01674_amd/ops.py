"""PyTorch-facing calls of the SG-WLS library.

Torch supplies device memory and the current HIP stream; every step of the
filter runs in the HIP kernels behind the C ABI (``include/sgwls.h``).  The
names follow the paper (Liu et al., ICCV 2017): ``lam`` is lambda of Eq. (1),
``r`` the neighbourhood radius, ``iters`` the iteration count T and ``stride``
the sliding step tau of Sec. 2.3; ``kind`` selects omega^exp or omega^frac of
Eq. (2).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, replace
from typing import Optional

import torch

from . import _native as nat

_KIND = {"exp": 0, "frac": 1}
_PREC = {"fp32": 0, "fp64_pivot": 1, "fp32_delta": 2, "auto": 3}
_PREC_NAME = {v: k for k, v in _PREC.items()}


@dataclass(frozen=True)
class Params:
    lam: float = 1.0
    r: int = 1
    iters: int = 1
    stride: int = 1
    kind: str = "exp"
    sigma_s: Optional[float] = None     # default: r (the paper's setting, Sec. 3)
    sigma_r: float = 0.1
    alpha_s: float = 1.2
    alpha_r: float = 1.2
    eps: float = 1e-4
    prec: str = "auto"      # float32 unless the host bound on lambda*omega asks for FP64 pivots

    def c(self) -> nat.SgwlsParams:
        if self.kind not in _KIND:
            raise ValueError(f"kind must be one of {list(_KIND)}")
        if self.prec not in _PREC:
            raise ValueError(f"prec must be one of {list(_PREC)}")
        ss = float(self.r) if self.sigma_s is None else float(self.sigma_s)
        return nat.SgwlsParams(float(self.lam), int(self.r), int(self.iters), int(self.stride),
                               _KIND[self.kind], ss, float(self.sigma_r), float(self.alpha_s),
                               float(self.alpha_r), float(self.eps), _PREC[self.prec])

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)


def params(**kw) -> Params:
    """Params from keyword arguments; unknown keys raise."""
    return Params(**kw)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(dev: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _image(x: torch.Tensor, name: str):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if x.dim() == 2:
        return 1, x.shape[0], x.shape[1]
    if x.dim() == 3:
        return x.shape[0], x.shape[1], x.shape[2]
    raise ValueError(f"{name} must be (M, N) or (C, M, N)")


def _guidance(g: torch.Tensor, M: int, N: int, dev: torch.device):
    _image(g, "g")
    if g.dim() != 2 or g.shape != (M, N):
        raise ValueError(f"g must be ({M}, {N})")
    if g.device != dev:
        raise ValueError("g must be on the same device as f")


def _lambda(lambda_dev: Optional[torch.Tensor], dev):
    if lambda_dev is None:
        return None
    if not lambda_dev.is_cuda or lambda_dev.dtype != torch.float32 or lambda_dev.numel() != 1:
        raise TypeError("lambda_dev must be a one-element float32 CUDA tensor")
    if lambda_dev.device != dev:
        raise ValueError("lambda_dev must be on the device of f")
    return lambda_dev


def resolve_precision(p: Params, want_lambda_grad: bool = False) -> str:
    """The precision a call with p runs in ("fp32", "fp64_pivot" or
    "fp32_delta"): p.prec unless it is "auto", which the library resolves
    from its bound on lambda * omega (and to "fp64_pivot" for a backward call
    that asks for the lambda gradient)."""
    return _PREC_NAME[int(nat.lib.sgwls_resolve_precision(ctypes.byref(p.c()), int(want_lambda_grad)))]


def workspace_bytes(C: int, M: int, N: int, p: Params, save_for_backward: bool = False) -> int:
    n = nat.lib.sgwls_workspace_bytes(C, M, N, ctypes.byref(p.c()), int(save_for_backward))
    if n == 0:
        nat.check(nat.lib.sgwls_validate(C, M, N, ctypes.byref(p.c())), "sgwls_workspace_bytes")
    return int(n)


def validate(C: int, M: int, N: int, p: Params) -> int:
    return int(nat.lib.sgwls_validate(C, M, N, ctypes.byref(p.c())))


def _workspace(nbytes: int, dev) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=dev)


def _seps_buffer(seps: torch.Tensor, dev) -> None:
    if seps.dtype != torch.uint8 or seps.device != dev or not seps.is_contiguous():
        raise ValueError("seps must be a contiguous uint8 tensor on the device of the images")


def sgwls_filter(f: torch.Tensor, g: torch.Tensor, p: Params, *,
                 lambda_dev: Optional[torch.Tensor] = None,
                 saved: Optional[torch.Tensor] = None,
                 out: Optional[torch.Tensor] = None,
                 workspace: Optional[torch.Tensor] = None,
                 seps: Optional[torch.Tensor] = None) -> torch.Tensor:
    """SG-WLS filter of f (C x M x N or M x N) guided by g (M x N), Sec. 2.3.

    ``saved`` (optional, 2T x C x M x N float32) receives every pass input for
    the backward call.  ``out`` may be f itself (in-place filtering).
    ``seps`` (optional, with saved; uint8, separator_bytes_nchw(1, C, M, N, p)
    bytes) receives every pass's separator solutions for the backward; then
    saved[0] is not written (the backward takes f itself, so ``out`` must
    not be f)."""
    C, M, N = _image(f, "f")
    dev = f.device
    _guidance(g, M, N, dev)
    lam = _lambda(lambda_dev, dev)
    if out is None:
        out = torch.empty_like(f)
    elif out.shape != f.shape or out.dtype != f.dtype or not out.is_contiguous() or out.device != dev:
        raise ValueError("out must match f")
    if saved is not None:
        if (saved.dtype != torch.float32 or not saved.is_contiguous() or saved.device != dev
                or saved.numel() != 2 * p.iters * C * M * N):
            raise ValueError("saved must be a contiguous float32 tensor of 2T*C*M*N elements")
    nbytes = workspace_bytes(C, M, N, p, saved is not None)
    ws = workspace if workspace is not None else _workspace(nbytes, dev)
    if ws.numel() < nbytes or ws.device != dev:
        raise ValueError("workspace too small")
    cp = p.c()
    if seps is not None:
        _seps_buffer(seps, dev)
        nat.check(nat.lib.sgwls_filter_nchw_seps(_ptr(f), _ptr(g), _ptr(out), 1, C, M, N,
                                                 ctypes.byref(cp), _ptr(lam), _ptr(saved),
                                                 _ptr(seps), seps.numel(), _ptr(ws), ws.numel(),
                                                 _stream(dev)),
                  "sgwls_filter_nchw_seps")
        return out
    nat.check(nat.lib.sgwls_filter(_ptr(f), _ptr(g), _ptr(out), C, M, N, ctypes.byref(cp),
                                   _ptr(lam), _ptr(saved), _ptr(ws), ws.numel(), _stream(dev)),
              "sgwls_filter")
    return out


def filter_status(workspace: torch.Tensor) -> None:
    """Raise if a fused pass of an earlier filter call on ``workspace`` gave
    up a wait (its results are then undefined); synchronises the current
    stream.  Fused passes run only when SGWLS_ONE_LAUNCH is 1 or 2."""
    nat.check(nat.lib.sgwls_filter_status(_ptr(workspace), _stream(workspace.device)),
              "sgwls_filter_status")


def interpolate_workspace_bytes(C: int, M: int, N: int, p: Params) -> int:
    n = nat.lib.sgwls_interpolate_workspace_bytes(C, M, N, ctypes.byref(p.c()))
    if n == 0:
        raise ValueError("invalid interpolation arguments")
    return int(n)


def sgwls_interpolate(f: torch.Tensor, h: torch.Tensor, g: torch.Tensor, p: Params, *,
                      lambda_dev: Optional[torch.Tensor] = None,
                      out: Optional[torch.Tensor] = None,
                      workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Guided sparse interpolation of Eq. (21): S(f) / S(h), with f the sparse
    input (C x M x N or M x N, 0 where unknown), h the index map (M x N, 1
    where f is known) and S the SG-WLS filter guided by g."""
    C, M, N = _image(f, "f")
    dev = f.device
    _guidance(g, M, N, dev)
    _guidance(h, M, N, dev)
    lam = _lambda(lambda_dev, dev)
    if out is None:
        out = torch.empty_like(f)
    elif out.shape != f.shape or out.dtype != f.dtype or not out.is_contiguous() or out.device != dev:
        raise ValueError("out must match f")
    nbytes = interpolate_workspace_bytes(C, M, N, p)
    ws = workspace if workspace is not None else _workspace(nbytes, dev)
    if ws.numel() < nbytes or ws.device != dev:
        raise ValueError("workspace too small")
    nat.check(nat.lib.sgwls_interpolate(_ptr(f), _ptr(h), _ptr(g), _ptr(out), C, M, N,
                                        ctypes.byref(p.c()), _ptr(lam), _ptr(ws), ws.numel(),
                                        _stream(dev)),
              "sgwls_interpolate")
    return out


def wls2d_workspace_bytes(C: int, M: int, N: int, p: Params) -> int:
    n = nat.lib.sgwls_wls2d_workspace_bytes(C, M, N, ctypes.byref(p.c()))
    if n == 0:
        raise ValueError("invalid 2D WLS arguments (1 <= C <= 4)")
    return int(n)


def wls2d(f: torch.Tensor, g: torch.Tensor, p: Params, *, max_iters: int = 1000,
          tol: float = 1e-6, out: Optional[torch.Tensor] = None,
          workspace: Optional[torch.Tensor] = None):
    """The 2D WLS model SG-WLS approximates (Eqs. 1-4), solved by conjugate
    gradients on the GPU.  Returns (u, iterations, relative residual)."""
    C, M, N = _image(f, "f")
    dev = f.device
    _guidance(g, M, N, dev)
    if out is None:
        out = torch.empty_like(f)
    elif out.shape != f.shape or out.dtype != f.dtype or not out.is_contiguous() or out.device != dev:
        raise ValueError("out must match f")
    nbytes = wls2d_workspace_bytes(C, M, N, p)
    ws = workspace if workspace is not None else _workspace(nbytes, dev)
    if ws.numel() < nbytes or ws.device != dev:
        raise ValueError("workspace too small")
    its, rel = ctypes.c_int(0), ctypes.c_double(0.0)
    nat.check(nat.lib.sgwls_wls2d(_ptr(f), _ptr(g), _ptr(out), C, M, N, ctypes.byref(p.c()),
                                  int(max_iters), float(tol), ctypes.byref(its),
                                  ctypes.byref(rel), _ptr(ws), ws.numel(), _stream(dev)),
              "sgwls_wls2d")
    return out, its.value, rel.value


def sgwls_pass(direction: int, x: torch.Tensor, g: torch.Tensor, p: Params, *,
               lambda_dev: Optional[torch.Tensor] = None,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One pass of Sec. 2.3: direction 0 = column direction, 1 = row direction."""
    C, M, N = _image(x, "x")
    dev = x.device
    _guidance(g, M, N, dev)
    lam = _lambda(lambda_dev, dev)
    out = torch.empty_like(x) if out is None else out
    nbytes = workspace_bytes(C, M, N, p)
    ws = _workspace(nbytes, dev)
    cp = p.c()
    nat.check(nat.lib.sgwls_pass(int(direction), _ptr(x), _ptr(g), _ptr(out), C, M, N,
                                 ctypes.byref(cp), _ptr(lam), _ptr(ws), ws.numel(), _stream(dev)),
              "sgwls_pass")
    return out


def sgwls_pass_stages(stages: int, direction: int, x: torch.Tensor, g: torch.Tensor, p: Params, *,
                      lambda_dev: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                      workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """The stages of one pass (see sgwls_pass_stages in sgwls.h): mask bits
    1 reduce, 2 interface, 4 expand, 8 transposed output.  With a shared
    workspace and one channel block (C = 1 or 3), masks 1, 2 and 4 called in
    order compute one pass."""
    C, M, N = _image(x, "x")
    dev = x.device
    _guidance(g, M, N, dev)
    lam = _lambda(lambda_dev, dev)
    if out is None:
        out = torch.empty_like(x)
    nbytes = workspace_bytes(C, M, N, p)
    ws = workspace if workspace is not None else _workspace(nbytes, dev)
    if ws.numel() < nbytes or ws.device != dev:
        raise ValueError("workspace too small")
    nat.check(nat.lib.sgwls_pass_stages(int(stages), int(direction), _ptr(x), _ptr(g), _ptr(out), C, M,
                                        N, ctypes.byref(p.c()), _ptr(lam), _ptr(ws), ws.numel(),
                                        _stream(dev)),
              "sgwls_pass_stages")
    return out


# ---------------------------------------------------------------------------
# Gradients.

def backward_workspace_bytes(C: int, M: int, N: int, p: Params) -> int:
    n = nat.lib.sgwls_backward_workspace_bytes(C, M, N, ctypes.byref(p.c()))
    if n == 0:
        nat.check(nat.lib.sgwls_validate(C, M, N, ctypes.byref(p.c())), "sgwls_backward_workspace_bytes")
    return int(n)


def _grad_lambda_buffer(grad_lambda: Optional[torch.Tensor], dev):
    if grad_lambda is None:
        return None
    if (not grad_lambda.is_cuda or grad_lambda.dtype != torch.float64 or grad_lambda.numel() != 1
            or grad_lambda.device != dev):
        raise TypeError("grad_lambda must be a one-element float64 tensor on the device of f")
    return grad_lambda


def sgwls_pass_backward(direction: int, x: torch.Tensor, g: torch.Tensor, ybar: torch.Tensor,
                        p: Params, *, lambda_dev: Optional[torch.Tensor] = None,
                        want_g: bool = True, want_lambda: bool = True):
    """Adjoint of one pass (column direction 0, row direction 1): returns
    (xbar, gbar or None, grad_lambda (float64 device tensor) or None)."""
    C, M, N = _image(x, "x")
    dev = x.device
    _guidance(g, M, N, dev)
    if _image(ybar, "ybar") != (C, M, N):
        raise ValueError("ybar must match x")
    lam = _lambda(lambda_dev, dev)
    xbar = torch.empty_like(x)
    gbar = torch.empty_like(g) if want_g else None
    glam = torch.empty(1, dtype=torch.float64, device=dev) if want_lambda else None
    ws = _workspace(backward_workspace_bytes(C, M, N, p), dev)
    nat.check(nat.lib.sgwls_pass_backward(int(direction), _ptr(x), _ptr(g), _ptr(ybar), _ptr(xbar),
                                          _ptr(gbar), _ptr(glam), C, M, N, ctypes.byref(p.c()),
                                          _ptr(lam), _ptr(ws), ws.numel(), _stream(dev)),
              "sgwls_pass_backward")
    return xbar, gbar, glam


def sgwls_backward(g: torch.Tensor, saved: torch.Tensor, grad_u: torch.Tensor, p: Params, *,
                   lambda_dev: Optional[torch.Tensor] = None, want_g: bool = True,
                   want_lambda: bool = True, grad_f: Optional[torch.Tensor] = None,
                   grad_g: Optional[torch.Tensor] = None,
                   grad_lambda: Optional[torch.Tensor] = None,
                   workspace: Optional[torch.Tensor] = None,
                   seps: Optional[torch.Tensor] = None, f: Optional[torch.Tensor] = None):
    """Adjoint of ``sgwls_filter`` given the pass inputs it saved: returns
    (grad_f, grad_g or None, grad_lambda (float64 device tensor) or None).
    ``seps``: the separators that filter call kept (p must be its p), with
    ``f`` its input (pass 0's input, which that call did not copy)."""
    C, M, N = _image(grad_u, "grad_u")
    dev = grad_u.device
    _guidance(g, M, N, dev)
    if (saved.dtype != torch.float32 or not saved.is_contiguous() or saved.device != dev
            or saved.numel() != 2 * p.iters * C * M * N):
        raise ValueError("saved must be a contiguous float32 tensor of 2T*C*M*N elements")
    lam = _lambda(lambda_dev, dev)
    if grad_f is None:
        grad_f = torch.empty_like(grad_u)
    elif grad_f.shape != grad_u.shape or grad_f.dtype != torch.float32 or not grad_f.is_contiguous():
        raise ValueError("grad_f must match grad_u")
    if want_g:
        gbar = torch.empty_like(g) if grad_g is None else grad_g
        if gbar.shape != g.shape or gbar.dtype != torch.float32 or not gbar.is_contiguous():
            raise ValueError("grad_g must match g")
    else:
        gbar = None
    if want_lambda:
        glam = (torch.empty(1, dtype=torch.float64, device=dev) if grad_lambda is None
                else _grad_lambda_buffer(grad_lambda, dev))
    else:
        glam = None
    nbytes = backward_workspace_bytes(C, M, N, p)
    ws = workspace if workspace is not None else _workspace(nbytes, dev)
    if ws.numel() < nbytes or ws.device != dev:
        raise ValueError("workspace too small")
    if seps is not None:
        _seps_buffer(seps, dev)
        if f is None or f.shape != grad_u.shape or f.dtype != torch.float32 or not f.is_contiguous():
            raise ValueError("f (the filter call's input) must come with seps")
        nat.check(nat.lib.sgwls_backward_nchw_seps(_ptr(g), _ptr(f), _ptr(saved), _ptr(seps),
                                                   seps.numel(), _ptr(grad_u), _ptr(grad_f),
                                                   _ptr(gbar), _ptr(glam), 1, C, M, N,
                                                   ctypes.byref(p.c()), _ptr(lam), _ptr(ws),
                                                   ws.numel(), _stream(dev)),
                  "sgwls_backward_nchw_seps")
        return grad_f, gbar, glam
    nat.check(nat.lib.sgwls_backward(_ptr(g), _ptr(saved), _ptr(grad_u), _ptr(grad_f), _ptr(gbar),
                                     _ptr(glam), C, M, N, ctypes.byref(p.c()), _ptr(lam), _ptr(ws),
                                     ws.numel(), _stream(dev)),
              "sgwls_backward")
    return grad_f, gbar, glam


def _batch4(x: torch.Tensor, name: str):
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float32:
        raise TypeError(f"{name} must be a float32 CUDA (HIP) tensor")
    if not x.is_contiguous() or x.dim() != 4:
        raise ValueError(f"{name} must be a contiguous (B, C, M, N) tensor")
    return tuple(x.shape)


def workspace_bytes_nchw(B: int, C: int, M: int, N: int, p: Params,
                         save_for_backward: bool = False) -> int:
    """Workspace bytes of sgwls_filter_nchw over B images of C x M x N."""
    n = nat.lib.sgwls_workspace_bytes_nchw(B, C, M, N, ctypes.byref(p.c()), int(save_for_backward))
    if n == 0:
        raise ValueError("invalid batch or parameters")
    return int(n)


def separator_bytes_nchw(B: int, C: int, M: int, N: int, p: Params) -> int:
    """Bytes of the saved-separator buffer of B images of C x M x N (0: the
    case has no saved-separator path)."""
    return int(nat.lib.sgwls_separator_bytes_nchw(B, C, M, N, ctypes.byref(p.c())))


def sgwls_filter_nchw(f: torch.Tensor, g: torch.Tensor, p: Params, *,
                      lambda_dev: Optional[torch.Tensor] = None,
                      saved: Optional[torch.Tensor] = None,
                      seps: Optional[torch.Tensor] = None,
                      out: Optional[torch.Tensor] = None,
                      workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """The filter of B equal-shape images in each launch: f (B, C, M, N), g
    (B, M, N); saved (optional) B x 2T x C x M x N; seps (optional, with
    saved): a uint8 device tensor of separator_bytes_nchw bytes that receives
    every pass's separator solutions for sgwls_backward_nchw (saved[:, 0] is
    then not written: the backward takes f itself, so ``out`` must not be
    f)."""
    B, C, M, N = _batch4(f, "f")
    dev = f.device
    if g.shape != (B, M, N) or not g.is_contiguous() or g.dtype != torch.float32 or g.device != dev:
        raise ValueError(f"g must be a contiguous float32 ({B}, {M}, {N}) tensor on the device of f")
    lam = _lambda(lambda_dev, dev)
    out = torch.empty_like(f) if out is None else out
    if out.shape != f.shape or not out.is_contiguous() or out.device != dev:
        raise ValueError("out must match f")
    if saved is not None and (saved.numel() != B * 2 * p.iters * C * M * N or not saved.is_contiguous()
                              or saved.dtype != torch.float32 or saved.device != dev):
        raise ValueError("saved must be a contiguous float32 tensor of B*2T*C*M*N elements")
    nbytes = nat.lib.sgwls_workspace_bytes_nchw(B, C, M, N, ctypes.byref(p.c()), int(saved is not None))
    if nbytes == 0:
        nat.check(nat.lib.sgwls_validate(C, M, N, ctypes.byref(p.c())) or 4, "sgwls_workspace_bytes_nchw")
    ws = workspace if workspace is not None else _workspace(nbytes, dev)
    if ws.numel() < nbytes or ws.device != dev:
        raise ValueError("workspace too small")
    if seps is not None:
        _seps_buffer(seps, dev)
        nat.check(nat.lib.sgwls_filter_nchw_seps(_ptr(f), _ptr(g), _ptr(out), B, C, M, N,
                                                 ctypes.byref(p.c()), _ptr(lam), _ptr(saved),
                                                 _ptr(seps), seps.numel(), _ptr(ws), ws.numel(),
                                                 _stream(dev)),
                  "sgwls_filter_nchw_seps")
        return out
    nat.check(nat.lib.sgwls_filter_nchw(_ptr(f), _ptr(g), _ptr(out), B, C, M, N, ctypes.byref(p.c()),
                                        _ptr(lam), _ptr(saved), _ptr(ws), ws.numel(), _stream(dev)),
              "sgwls_filter_nchw")
    return out


def sgwls_backward_nchw(g: torch.Tensor, saved: torch.Tensor, grad_u: torch.Tensor, p: Params, *,
                        lambda_dev: Optional[torch.Tensor] = None, want_g: bool = True,
                        want_lambda: bool = True, workspace: Optional[torch.Tensor] = None,
                        seps: Optional[torch.Tensor] = None, f: Optional[torch.Tensor] = None):
    """Adjoint of sgwls_filter_nchw: returns (grad_f (B, C, M, N), grad_g
    (B, M, N) or None, grad_lambda summed over the batch (float64 device
    tensor) or None).  seps: the separators the forward kept (then p must be
    the forward's, the call runs in the forward's precision, and f is the
    forward's input, pass 0's input, which that call did not copy)."""
    B, C, M, N = _batch4(grad_u, "grad_u")
    dev = grad_u.device
    lam = _lambda(lambda_dev, dev)
    grad_f = torch.empty_like(grad_u)
    gbar = torch.empty_like(g) if want_g else None
    glam = torch.empty(1, dtype=torch.float64, device=dev) if want_lambda else None
    nbytes = nat.lib.sgwls_backward_workspace_bytes_nchw(B, C, M, N, ctypes.byref(p.c()))
    ws = workspace if workspace is not None else _workspace(nbytes, dev)
    if ws.numel() < nbytes or ws.device != dev:
        raise ValueError("workspace too small")
    if seps is not None:
        _seps_buffer(seps, dev)
        if f is None or f.shape != grad_u.shape or f.dtype != torch.float32 or not f.is_contiguous():
            raise ValueError("f (the filter call's input) must come with seps")
        nat.check(nat.lib.sgwls_backward_nchw_seps(_ptr(g), _ptr(f), _ptr(saved), _ptr(seps),
                                                   seps.numel(), _ptr(grad_u), _ptr(grad_f),
                                                   _ptr(gbar), _ptr(glam), B, C, M, N,
                                                   ctypes.byref(p.c()), _ptr(lam), _ptr(ws),
                                                   ws.numel(), _stream(dev)),
                  "sgwls_backward_nchw_seps")
        return grad_f, gbar, glam
    nat.check(nat.lib.sgwls_backward_nchw(_ptr(g), _ptr(saved), _ptr(grad_u), _ptr(grad_f), _ptr(gbar),
                                          _ptr(glam), B, C, M, N, ctypes.byref(p.c()), _ptr(lam),
                                          _ptr(ws), ws.numel(), _stream(dev)),
              "sgwls_backward_nchw")
    return grad_f, gbar, glam


class SGWLSFunction(torch.autograd.Function):
    """u = SG-WLS(f, g, lambda) with gradients for f, g and lambda.

    f: (C, M, N) or (B, C, M, N) float32; g: (M, N) or (B, M, N) float32;
    lam: one-element float32 tensor on the device (a learnable scalar).  The
    forward pass saves every pass input (2T images per image) and, where the
    case has that path, every pass's separator solutions; the backward pass
    runs the adjoint kernels, which recompute the weights from g (and, with
    saved separators, solve only the adjoint's separator systems).  A batch
    runs as one NCHW call each way (every launch covers all images).  The
    environment variable SGWLS_SAVE_SEPARATORS=0 turns the separators off."""

    @staticmethod
    def forward(ctx, f, g, lam, p: Params):
        batched = f.dim() == 4
        fb = f.contiguous() if batched else f.contiguous().unsqueeze(0)
        gb = g.contiguous() if batched else g.contiguous().unsqueeze(0)
        if fb.dim() != 4 or gb.dim() != 3 or gb.shape[0] != fb.shape[0]:
            raise ValueError("f must be (C,M,N) or (B,C,M,N) with g (M,N) or (B,M,N)")
        B, C, M, N = fb.shape
        lam_dev = lam.detach().reshape(1).to(torch.float32).contiguous()
        if p.prec == "auto":
            # The automatic precision is decided here, once for the forward and
            # the backward.  A lambda that needs a gradient asks for FP64 pivots
            # in both calls whatever its value (no host sync); otherwise the
            # bound on lambda * omega decides, from lambda read back once.
            if ctx.needs_input_grad[2]:
                p = p.with_(prec="fp64_pivot")
            else:
                p = p.with_(lam=max(float(lam_dev.item()), 0.0))
                p = p.with_(prec=resolve_precision(p, False))
        saved = torch.empty((B, 2 * p.iters, C, M, N), dtype=torch.float32, device=f.device)
        nsep = separator_bytes_nchw(B, C, M, N, p) if os.environ.get("SGWLS_SAVE_SEPARATORS", "1") != "0" else 0
        seps = torch.empty(nsep, dtype=torch.uint8, device=f.device) if nsep > 0 else None
        out = sgwls_filter_nchw(fb, gb, p, lambda_dev=lam_dev, saved=saved, seps=seps)
        ctx.p = p
        ctx.batched = batched
        ctx.lam_shape = lam.shape
        ctx.has_seps = seps is not None
        if seps is None:
            ctx.save_for_backward(gb, saved, lam_dev)
        else:
            # pass 0's input is f itself (not copied into saved)
            ctx.save_for_backward(gb, saved, lam_dev, seps, fb)
        return out if batched else out[0]

    @staticmethod
    def backward(ctx, grad_out):
        gb, saved, lam_dev = ctx.saved_tensors[:3]
        seps = ctx.saved_tensors[3] if ctx.has_seps else None
        fb = ctx.saved_tensors[4] if ctx.has_seps else None
        p = ctx.p
        go = grad_out.contiguous() if ctx.batched else grad_out.contiguous().unsqueeze(0)
        want_f, want_g, want_l = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        grad_f, grad_g, glam = sgwls_backward_nchw(gb, saved, go, p, lambda_dev=lam_dev,
                                                   want_g=want_g, want_lambda=want_l, seps=seps,
                                                   f=fb)
        gl_out = glam.to(torch.float32).reshape(ctx.lam_shape) if want_l else None
        if not ctx.batched:
            grad_f = grad_f[0]
            grad_g = grad_g[0] if want_g else None
        return (grad_f if want_f else None), grad_g, gl_out, None


def sgwls(f: torch.Tensor, g: torch.Tensor, lam: torch.Tensor, p: Params) -> torch.Tensor:
    """Differentiable SG-WLS filter (see SGWLSFunction); p.lam is ignored in
    favour of the tensor lam."""
    return SGWLSFunction.apply(f, g, lam, p)


# ---------------------------------------------------------------------------
# Batches of uneven images.

def _batch_args(fs, gs, ps, outs):
    B = len(fs)
    if B < 1 or len(gs) != B or len(ps) != B or (outs is not None and len(outs) != B):
        raise ValueError("fs, gs, ps (and outs) must be non-empty lists of equal length")
    imgs = (nat.SgwlsImage * B)()
    cps = (nat.SgwlsParams * B)()
    dev = fs[0].device
    res = []
    for b in range(B):
        C, M, N = _image(fs[b], f"fs[{b}]")
        if fs[b].device != dev:
            raise ValueError("all images must be on one device")
        _guidance(gs[b], M, N, dev)
        u = torch.empty_like(fs[b]) if outs is None else outs[b]
        if u.shape != fs[b].shape or u.dtype != torch.float32 or not u.is_contiguous() or u.device != dev:
            raise ValueError(f"outs[{b}] must match fs[{b}]")
        imgs[b] = nat.SgwlsImage(fs[b].data_ptr(), gs[b].data_ptr(), u.data_ptr(), C, M, N)
        cps[b] = ps[b].c()
        res.append(u)
    return imgs, cps, B, dev, res


def batched_workspace_bytes(fs, gs, ps) -> int:
    imgs, cps, B, _, _ = _batch_args(fs, gs, ps, list(fs))
    n = nat.lib.sgwls_batched_workspace_bytes(imgs, cps, B)
    if n == 0:
        raise nat.SgwlsError(1, "sgwls_batched_workspace_bytes: invalid batch")
    return int(n)


def sgwls_filter_batched(fs, gs, ps, *, outs=None, variant: Optional[int] = None,
                         workspace: Optional[torch.Tensor] = None, stream=None):
    """Filter a list of images (each (C, M, N) or (M, N) float32) with their
    guidance images and per-image Params in one batched call.  On a
    non-default stream the call is captured into a hipGraph once and replayed
    by identical later calls.  Returns the list of outputs."""
    imgs, cps, B, dev, outs = _batch_args(fs, gs, ps, outs)
    nbytes = nat.lib.sgwls_batched_workspace_bytes(imgs, cps, B)
    if nbytes == 0:
        nat.check(nat.lib.sgwls_filter_batched_variant(imgs, cps, B, -1, None, 0, None),
                  "sgwls_filter_batched")
    ws = workspace if workspace is not None else _workspace(nbytes, dev)
    if ws.numel() < nbytes or ws.device != dev:
        raise ValueError("workspace too small")
    st = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream(dev)
    nat.check(nat.lib.sgwls_filter_batched_variant(imgs, cps, B, -1 if variant is None else int(variant),
                                                   _ptr(ws), ws.numel(), st),
              "sgwls_filter_batched")
    return outs


def batched_variant_count(prec: str = "fp32") -> int:
    return int(nat.lib.sgwls_batched_variant_count(_PREC[prec]))


def autotune_batched(fs, gs, ps, reps: int = 3, workspace: Optional[torch.Tensor] = None) -> int:
    """Time every batched variant on this batch and keep the fastest for its
    precision, weight kind and total size; returns the chosen variant."""
    imgs, cps, B, dev, _ = _batch_args(fs, gs, ps, None)
    nbytes = batched_workspace_bytes(fs, gs, ps)
    ws = workspace if workspace is not None else _workspace(nbytes, dev)
    chosen = ctypes.c_int(-1)
    nat.check(nat.lib.sgwls_autotune_batched(imgs, cps, B, _ptr(ws), ws.numel(), _stream(dev),
                                             int(reps), ctypes.byref(chosen)),
              "sgwls_autotune_batched")
    return int(chosen.value)


def batched_graph_count() -> int:
    return int(nat.lib.sgwls_batched_graph_count())


def batched_graph_clear() -> None:
    nat.lib.sgwls_batched_graph_clear()


# ---------------------------------------------------------------------------
# Kernel variants and autotuning (stride-1 passes).

def variant_count(r: int, channel_block: int, prec: str = "fp32") -> int:
    return int(nat.lib.sgwls_variant_count(int(r), int(channel_block), _PREC[prec]))


def tune_pin(direction: int, channel_block: int, M: int, N: int, p: Params, variant: int) -> None:
    nat.check(nat.lib.sgwls_tune_pin(int(direction), int(channel_block), int(M), int(N),
                                     ctypes.byref(p.c()), int(variant)), "sgwls_tune_pin")


def tune_query(direction: int, channel_block: int, M: int, N: int, p: Params) -> int:
    return int(nat.lib.sgwls_tune_query(int(direction), int(channel_block), int(M), int(N),
                                        ctypes.byref(p.c())))


def tune_clear() -> None:
    nat.lib.sgwls_tune_clear()


def device_arch(dev=None) -> str:
    name = torch.cuda.get_device_properties(dev or torch.cuda.current_device()).gcnArchName
    return name.split(":")[0]


def autotune(f: torch.Tensor, g: torch.Tensor, p: Params, reps: int = 10):
    """Time every compiled kernel variant of both pass directions on this image
    and keep the fastest for its shape (synchronises the current stream).
    Returns {(direction, channel_block): variant}."""
    C, M, N = _image(f, "f")
    dev = f.device
    _guidance(g, M, N, dev)
    y = torch.empty_like(f)
    ws = _workspace(workspace_bytes(C, M, N, p), dev)
    chosen = (ctypes.c_int * 4)()
    nat.check(nat.lib.sgwls_autotune(_ptr(f), _ptr(g), _ptr(y), C, M, N, ctypes.byref(p.c()),
                                     _ptr(ws), ws.numel(), _stream(dev), int(reps), chosen),
              "sgwls_autotune")
    out = {}
    for d in (0, 1):
        for i, cb in enumerate((3, 1)):
            if chosen[2 * d + i] >= 0:
                out[(d, cb)] = chosen[2 * d + i]
    return out


def tune_save(path: str, arch: Optional[str] = None) -> None:
    nat.check(nat.lib.sgwls_tune_save(path.encode(), (arch or device_arch()).encode()),
              "sgwls_tune_save")


def tune_load(path: str, arch: Optional[str] = None) -> bool:
    """Merge a saved tuning table; False (table unchanged) if the file is
    missing, malformed, or from another library version or architecture."""
    return nat.lib.sgwls_tune_load(path.encode(), (arch or device_arch()).encode()) == 0
