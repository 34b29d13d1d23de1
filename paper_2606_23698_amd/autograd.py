"""Differentiable Ozaki-Bailey 3-D FFT.

The forward transform is linear, Y = F X, so the vector-Jacobian product is
the Hermitian adjoint, grad_X = F^H grad_Y = conj(F conj(grad_Y)), which the
library computes with the conjugate roots through the same emulated kernels
(fft3d_z2z_adjoint).  PyTorch's complex autograd convention (gradients are
conjugate Wirtinger derivatives) makes this the exact backward of a real loss.
"""
import torch

from . import api


class FFT3(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, substrate="auto"):
        plan = api.get_plan(x.shape, "fp64", substrate, x.device.index)
        ctx.plan = plan
        return plan.forward(x.contiguous())

    @staticmethod
    def backward(ctx, grad_y):
        return ctx.plan.adjoint(grad_y.contiguous()), None


class IFFT3(torch.autograd.Function):
    """Normalised inverse; its backward is the adjoint scaled by 1/(n1 n2 n3)."""

    @staticmethod
    def forward(ctx, y, substrate="auto"):
        plan = api.get_plan(y.shape, "fp64", substrate, y.device.index)
        ctx.plan = plan
        return plan.inverse(y.contiguous())

    @staticmethod
    def backward(ctx, grad_x):
        n = grad_x.numel()
        g = ctx.plan.forward(grad_x.contiguous())
        return g / n, None


def fft3(x, substrate="auto"):
    return FFT3.apply(x, substrate)


def ifft3(y, substrate="auto"):
    return IFFT3.apply(y, substrate)


def spectral_weights(shape, device, dtype=torch.float64):
    """w_k = 1 / (1 + |k|^2) with signed integer wavenumbers (fftfreq * n) per axis."""
    ks = [torch.fft.fftfreq(n, d=1.0 / n, dtype=dtype, device=device) for n in shape]
    k1, k2, k3 = torch.meshgrid(*ks, indexing="ij")
    return 1.0 / (1.0 + k1 * k1 + k2 * k2 + k3 * k3)


def spectral_loss(x, w, substrate="auto"):
    """L(x) = sum |w * FFT3(x)|^2."""
    y = fft3(x, substrate)
    return torch.sum(torch.abs(w * y) ** 2)
