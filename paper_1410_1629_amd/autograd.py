"""torch.autograd interface of the life cycle: images as a differentiable
function of the cell densities.

Forward calls run_photons; backward calls backward_density, which replays
every package from its random numbers and accumulates the detached
(score-function) derivative of the images with respect to the density of
each cell (the derivative of the reweighted estimator whose paths are held
fixed).  Both run entirely in the HIP kernels.  The absorbed-luminosity
tally is not differentiated.
"""
import torch

from . import binding


class RTImage(torch.autograd.Function):
    """images = RTImage.apply(rho, prob): rho is the device density tensor
    (float64 for the FP64 path, float32 for the FP32 traversal), prob the
    problem dict of `workloads`.  Returns the FP64 images
    [comp][n_lambda][pixels]."""

    @staticmethod
    def forward(ctx, rho, prob):
        p = dict(prob, flags=int(prob.get("flags", 7)) & ~binding.ABSORB)
        images = torch.empty(binding.image_shape(p), dtype=torch.float64, device=rho.device)
        binding.run_photons(p, rho.contiguous(), images, None, stats=False)
        ctx.prob = p
        ctx.save_for_backward(rho)
        return images

    @staticmethod
    def backward(ctx, grad_images):
        (rho,) = ctx.saved_tensors
        grad = torch.empty(rho.numel(), dtype=torch.float64, device=rho.device)
        binding.backward_density(ctx.prob, rho.contiguous(), grad_images.contiguous().to(torch.float64), grad,
                                 stats=False)
        return grad.to(rho.dtype).view_as(rho), None


def render(prob, rho):
    """Differentiable images of the problem at density `rho`."""
    return RTImage.apply(rho, prob)
