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
min_x ||H^H x - s||^2 with these operators.  FP32 plans with the
pixel-per-lane back-projection (the adjoint's requirement).
"""
from __future__ import annotations

from typing import List, Tuple

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


def refine(geom: Geometry, grid, echo, steps: int = 10, x0=None, method: str = "cg",
           **opts) -> Tuple[object, List[float]]:
    """Least-squares refinement of an image-shaped scene x for
    min_x ||H^H x - s||^2, starting from x0 (default: zero).

    method "cg": conjugate gradients on the normal equations (CGNR) with the
    operators applied directly; "sd": steepest descent with the gradient
    from autograd (loss.backward() through ``echo_model``) and the exact line
    search of a quadratic.  Returns x and the residual norms ||H^H x - s||
    before each step and after the last."""
    s = echo.contiguous()
    shape = (geom.n_scan, grid.ny, grid.nx)
    x = torch.zeros(shape, dtype=torch.complex64, device=s.device) if x0 is None else x0.clone()
    history = []
    if method == "cg":
        r = s - adjoint_hybrid(geom, grid, x, **opts)
        z = reconstruct_hybrid(geom, grid, r, **opts)
        p = z.clone()
        zz = _norm2(z)
        history.append(_norm2(r) ** 0.5)
        for _ in range(steps):
            w = adjoint_hybrid(geom, grid, p, **opts)
            ww = _norm2(w)
            if ww == 0.0 or zz == 0.0:
                break
            alpha = zz / ww
            x = x + alpha * p
            r = r - alpha * w
            z = reconstruct_hybrid(geom, grid, r, **opts)
            zz_new = _norm2(z)
            p = z + (zz_new / zz) * p
            zz = zz_new
            history.append(_norm2(r) ** 0.5)
        return x, history
    if method == "sd":
        for _ in range(steps):
            xv = x.detach().requires_grad_(True)
            res = echo_model(geom, grid, xv, **opts) - s
            loss = torch.sum(res.real ** 2 + res.imag ** 2)
            loss.backward()
            g = xv.grad.detach()            # 2 H (H^H x - s)
            history.append(float(loss.detach()) ** 0.5)
            ag = adjoint_hybrid(geom, grid, g, **opts)
            den = 2.0 * _norm2(ag)
            if den == 0.0:
                break
            x = x.detach() - (_norm2(g) / den) * g
        res = adjoint_hybrid(geom, grid, x, **opts) - s
        history.append(_norm2(res) ** 0.5)
        return x, history
    raise ValueError("method must be 'cg' or 'sd'")
