"""Differentiable hybrid reconstruction and its adjoint echo model.

The imaging operator H (echo -> image, ``reconstruct_hybrid``) is linear, and
``adjoint_hybrid`` evaluates its hand-written adjoint H^H (image -> echo).
Two torch.autograd.Functions pair them:

* ``reconstruct(geom, grid, echo)``: g = H s, backward H^H;
* ``echo_model(geom, grid, image)``: s = H^H x, backward H -- the forward echo
  model of a scene given as an image-shaped reflectivity x.

PyTorch's convention for complex tensors (the gradient of a real loss is the
conjugate Wirtinger derivative times 2) makes the backward of a linear map A
the adjoint A^H applied to the incoming gradient, so both functions compose
with ordinary autograd losses.  ``refine`` runs least-squares refinement
min_x ||H^H x - s||^2 with these operators (``refine_with`` for any linear
operator pair), with optional checkpoints of the iterate.  FP32 plans with the
pixel-per-lane back-projection (the adjoint's requirement).
"""
from __future__ import annotations

import os
from typing import Callable, List, Optional, Tuple

from . import Geometry, adjoint_hybrid, reconstruct_hybrid, _torch

torch = _torch()


class Reconstruct(torch.autograd.Function):
    """g = H s (hybrid reconstruction); backward: H^H."""

    @staticmethod
    def forward(ctx, echo, geom, grid, opts):
        ctx.geom, ctx.grid, ctx.opts = geom, grid, opts
        return reconstruct_hybrid(geom, grid, echo.contiguous(), **opts)

    @staticmethod
    def backward(ctx, grad):
        return adjoint_hybrid(ctx.geom, ctx.grid, grad.contiguous(), **ctx.opts), None, None, None


class EchoModel(torch.autograd.Function):
    """s = H^H x (echo of an image-shaped scene); backward: H."""

    @staticmethod
    def forward(ctx, image, geom, grid, opts):
        ctx.geom, ctx.grid, ctx.opts = geom, grid, opts
        return adjoint_hybrid(geom, grid, image.contiguous(), **opts)

    @staticmethod
    def backward(ctx, grad):
        return reconstruct_hybrid(ctx.geom, ctx.grid, grad.contiguous(), **ctx.opts), None, None, None


def reconstruct(geom: Geometry, grid, echo, **opts):
    return Reconstruct.apply(echo, geom, grid, opts)


def echo_model(geom: Geometry, grid, image, **opts):
    return EchoModel.apply(image, geom, grid, opts)


def _norm2(t) -> float:
    return float(torch.linalg.vector_norm(t.reshape(-1).to(torch.complex128)) ** 2)


def _dot(a, b) -> complex:
    return complex(torch.vdot(a.reshape(-1).to(torch.complex128), b.reshape(-1).to(torch.complex128)))


def _save(path: str, state: dict) -> None:
    tmp = path + ".tmp"
    torch.save(state, tmp)
    os.replace(tmp, path)


def refine_with(apply_adj: Callable, apply_fwd: Callable, s, shape, steps: int = 10, x0=None, method: str = "cg",
                model: Optional[Callable] = None, checkpoint: Optional[str] = None,
                resume: bool = False) -> Tuple[object, List[float]]:
    """Least-squares refinement min_x ||A x - s||^2 for a linear echo model
    A = ``apply_adj`` (image-shaped x -> echo) with adjoint A^H =
    ``apply_fwd`` (echo -> image), from x0 (default zero).

    method "cg": conjugate gradients on the normal equations (CGNR);
    "sd": steepest descent with the gradient from autograd through
    ``model`` (a differentiable form of A) and the exact line search of a
    quadratic.  Returns x and the residual norms ||A x - s|| before each step
    and after the last.

    checkpoint: a .pt file written after every step with the iterate, the
    step index, the residual history and (CGNR) the recurrence's vectors;
    with resume=True an existing checkpoint of the same method is continued
    from its step, so an interrupted run ends where an uninterrupted one
    would.  Loaded with torch.load(weights_only=True)."""
    if method not in ("cg", "sd"):
        raise ValueError("method must be 'cg' or 'sd'")
    s = s.contiguous()
    state = None
    if checkpoint and resume and os.path.exists(checkpoint):
        state = torch.load(checkpoint, map_location=s.device, weights_only=True)
        if state.get("method") != method:
            raise ValueError(f"checkpoint {checkpoint} holds a {state.get('method')} run, not {method}")
    if method == "cg":
        if state is None:
            x = torch.zeros(shape, dtype=s.dtype, device=s.device) if x0 is None else x0.clone()
            r = s - apply_adj(x)
            z = apply_fwd(r)
            p = z.clone()
            zz = _norm2(z)
            history = [_norm2(r) ** 0.5]
            step = 0
        else:
            x, r, p, zz = state["x"], state["r"], state["p"], float(state["zz"])
            history, step = [float(h) for h in state["history"]], int(state["step"])
        while step < steps:
            w = apply_adj(p)
            ww = _norm2(w)
            if ww == 0.0 or zz == 0.0:
                break
            alpha = zz / ww
            x = x + alpha * p
            r = r - alpha * w
            z = apply_fwd(r)
            zz_new = _norm2(z)
            p = z + (zz_new / zz) * p
            zz = zz_new
            history.append(_norm2(r) ** 0.5)
            step += 1
            if checkpoint:
                _save(checkpoint, {"method": "cg", "step": step, "x": x, "r": r, "p": p, "zz": zz,
                                   "history": history})
        return x, history
    if model is None:
        raise ValueError("steepest descent needs a differentiable model")
    if state is None:
        x = torch.zeros(shape, dtype=s.dtype, device=s.device) if x0 is None else x0.clone()
        history, step = [], 0
    else:
        x, history, step = state["x"], [float(h) for h in state["history"]], int(state["step"])
    while step < steps:
        xv = x.detach().requires_grad_(True)
        res = model(xv) - s
        loss = torch.sum(res.real ** 2 + res.imag ** 2)
        loss.backward()
        g = xv.grad.detach()            # 2 A^H (A x - s)
        history.append(float(loss.detach()) ** 0.5)
        ag = apply_adj(g)
        den = 2.0 * _norm2(ag)
        if den == 0.0:
            break
        x = x.detach() - (_norm2(g) / den) * g
        step += 1
        if checkpoint:
            _save(checkpoint, {"method": "sd", "step": step, "x": x, "history": history})
    res = apply_adj(x) - s
    return x, history + [_norm2(res) ** 0.5]


def refine(geom: Geometry, grid, echo, steps: int = 10, x0=None, method: str = "cg", checkpoint: Optional[str] = None,
           resume: bool = False, **opts) -> Tuple[object, List[float]]:
    """Least-squares refinement of an image-shaped scene x for
    min_x ||H^H x - s||^2 with the library's operators (H^H the echo model
    ``adjoint_hybrid``, H ``reconstruct_hybrid``); see ``refine_with`` for
    the methods, the returned residual history and checkpoint / resume."""
    shape = (geom.n_scan, grid.ny, grid.nx)
    return refine_with(lambda x: adjoint_hybrid(geom, grid, x.contiguous(), **opts),
                       lambda r: reconstruct_hybrid(geom, grid, r.contiguous(), **opts), echo, shape, steps=steps,
                       x0=x0, method=method, model=lambda x: echo_model(geom, grid, x, **opts),
                       checkpoint=checkpoint, resume=resume)
