"""torch.autograd interface of the life cycle: images as a differentiable
function of the cell densities (RTImage), and of the densities, albedo, g
and source luminosities (RTImageOptics).

Forward calls run_photons; backward calls backward_density (or backward),
which replays every package from its random numbers and accumulates the
detached (score-function) derivative of the images -- the derivative of the
reweighted estimator whose paths are held fixed.  Both run entirely in the
HIP kernels.  When the run can keep an adjoint tape (binding.tape_bytes)
and it fits in a quarter of the free device memory, the forward run fills
one and the backward pass reads T and the peel-off contributions from it,
replaying each package once instead of twice (prob["adjoint_tape"] = False
turns this off).  prob["adjoint_estimator"] = "attached" makes RTImage's
backward pass the attached (pathwise) derivative instead (MCRT_ATTACHED:
random numbers fixed, scattering points moving with the densities; frames
and SED instruments; no tape).  These functions differentiate the images
only; a loss on the absorbed-luminosity tally goes through
binding.backward(adj_absorbed=).
"""
import numpy as np
import torch

from . import binding


def _attached(prob):
    est = prob.get("adjoint_estimator", "detached")
    if est not in ("detached", "attached"):
        raise ValueError("adjoint_estimator must be 'detached' or 'attached', not %r" % (est,))
    return est == "attached"


def _tape_for(prob, device):
    """A tape for the run, or None (not wanted, not possible, or too large)."""
    if not prob.get("adjoint_tape", True) or _attached(prob):
        return None
    n = binding.tape_bytes(prob)
    if n == 0:
        return None
    free, _ = torch.cuda.mem_get_info(device)
    return torch.empty(n, dtype=torch.uint8, device=device) if n < free // 4 else None


class RTImage(torch.autograd.Function):
    """images = RTImage.apply(rho, prob): rho is the device density tensor
    (float64 for the FP64 path, float32 for the FP32 traversal), prob the
    problem dict of `workloads`.  Returns the FP64 images
    [comp][n_lambda][pixels]."""

    @staticmethod
    def forward(ctx, rho, prob):
        p = dict(prob, flags=int(prob.get("flags", 7)) & ~binding.ABSORB)
        images = torch.empty(binding.image_shape(p), dtype=torch.float64, device=rho.device)
        tape = _tape_for(p, rho.device)
        binding.run_photons(p, rho.contiguous(), images, None, stats=False, tape=tape)
        ctx.prob = p
        ctx.tape = tape
        ctx.save_for_backward(rho)
        return images

    @staticmethod
    def backward(ctx, grad_images):
        (rho,) = ctx.saved_tensors
        grad = torch.empty(rho.numel(), dtype=torch.float64, device=rho.device)
        binding.backward_density(ctx.prob, rho.contiguous(), grad_images.contiguous().to(torch.float64), grad,
                                 stats=False, tape=ctx.tape, attached=_attached(ctx.prob))
        ctx.tape = None
        return grad.to(rho.dtype).view_as(rho), None


def render(prob, rho):
    """Differentiable images of the problem at density `rho`."""
    return RTImage.apply(rho, prob)


class RTImageOptics(torch.autograd.Function):
    """images = RTImageOptics.apply(rho, albedo, g, lum, prob): rho as in
    RTImage; albedo and g [n_lambda] and lum [n_src][n_lambda] FP64 tensors
    (their values replace the problem's; the library reads them on the
    host).  Gradients flow to every input that requires them, from one
    replay."""

    @staticmethod
    def forward(ctx, rho, albedo, g, lum, prob):
        if _attached(prob):
            raise ValueError("the attached estimator differentiates the densities only (use RTImage)")
        lum_h = lum.detach().to("cpu", torch.float64).numpy()
        p = dict(prob, flags=int(prob.get("flags", 7)) & ~binding.ABSORB,
                 albedo=albedo.detach().to("cpu", torch.float64).numpy().copy(),
                 g=g.detach().to("cpu", torch.float64).numpy().copy(),
                 sources=[dict(s, lum=np.array(lum_h[i])) for i, s in enumerate(prob["sources"])])
        images = torch.empty(binding.image_shape(p), dtype=torch.float64, device=rho.device)
        tape = _tape_for(p, rho.device)
        binding.run_photons(p, rho.contiguous(), images, None, stats=False, tape=tape)
        ctx.prob = p
        ctx.tape = tape
        ctx.save_for_backward(rho, albedo, g, lum)
        return images

    @staticmethod
    def backward(ctx, grad_images):
        rho, albedo, g, lum = ctx.saved_tensors
        need = ctx.needs_input_grad
        dev = rho.device
        outs = [torch.empty(t.numel(), dtype=torch.float64, device=dev) if need[i] else None
                for i, t in enumerate((rho, albedo, g, lum))]
        if not any(o is not None for o in outs):
            return None, None, None, None, None
        binding.backward(ctx.prob, rho.contiguous(), grad_images.contiguous().to(torch.float64), *outs, stats=False,
                         tape=ctx.tape)
        ctx.tape = None
        res = [None if o is None else o.to(t.dtype).view_as(t).to(t.device) for o, t in zip(outs, (rho, albedo, g, lum))]
        return res[0], res[1], res[2], res[3], None


def render_optics(prob, rho, albedo, g, lum):
    """Differentiable images of the problem at density `rho`, albedo and g
    per wavelength and source luminosities `lum` [n_src][n_lambda]."""
    return RTImageOptics.apply(rho, albedo, g, lum, prob)
