"""``TodChisq``: the TOD chi^2 as a differentiable torch function.

Forward calls ``tod_chisq`` (per-segment J, summed); backward calls the
hand-written adjoint ``tod_chisq_backward``.  Inputs that carry gradients:
maps [3][npix_total], per-segment gains [nseg], per-detector sigma0, f_knee,
alpha [ndet].  The decoded pointing, the TOD and n_corr are fixed inputs.
"""
import torch

from . import ops


class TodChisq(torch.autograd.Function):
    @staticmethod
    def forward(fctx, maps, gain, sigma0_det, fknee_det, alpha_det, problem):
        c, tod, prec, pix, psi, ncorr = problem
        det = torch.as_tensor(tod.seg_det_h, dtype=torch.long, device=maps.device)
        s0 = sigma0_det.detach().to(torch.float64)[det].contiguous()
        fk = fknee_det.detach().to(torch.float64)[det].contiguous()
        al = alpha_det.detach().to(torch.float64)[det].contiguous()
        g = gain.detach().to(torch.float64).contiguous()
        m = maps.detach().contiguous()
        out = torch.empty(tod.nseg, dtype=torch.float64, device=maps.device)
        c.tod_chisq(tod, prec, pix, psi, tod.d, ncorr, m, out, gain=g, sigma0=s0, fknee=fk, alpha=al)
        fctx.problem = problem
        fctx.save_for_backward(m, g, s0, fk, al)
        fctx.maps_dtype = maps.dtype
        return out.sum()

    @staticmethod
    def backward(fctx, gJ):
        c, tod, prec, pix, psi, ncorr = fctx.problem
        m, g, s0, fk, al = fctx.saved_tensors
        dev = m.device
        gm = torch.empty((3, tod.npix_total), dtype=torch.float64, device=dev)
        gg = torch.empty(tod.nseg, dtype=torch.float64, device=dev)
        gs = torch.empty(tod.ndet, dtype=torch.float64, device=dev)
        gf = torch.empty(tod.ndet, dtype=torch.float64, device=dev)
        ga = torch.empty(tod.ndet, dtype=torch.float64, device=dev)
        # the incoming gradient stays on the device: the adjoint kernels read it
        gj = gJ.detach().to(device=dev, dtype=torch.float64).reshape(1).contiguous()
        c.tod_chisq_backward(tod, prec, pix, psi, tod.d, ncorr, m, gj, gm, gg, gs, gf,
                             ga, gain=g, sigma0=s0, fknee=fk, alpha=al)
        return gm.to(fctx.maps_dtype), gg, gs, gf, ga, None


def tod_chisq(maps, gain, sigma0_det, fknee_det, alpha_det, ctx, tod, prec, pix, psi, ncorr):
    """Differentiable total chi^2 (see TodChisq)."""
    return TodChisq.apply(maps, gain, sigma0_det, fknee_det, alpha_det,
                          (ctx, tod, prec, pix, psi, ncorr))


def new_context(device=0):
    return ops.Context(device)
