"""Differentiable geodesic chains.

GeodesicChainFunction takes the gradient in one of two ways:
  method="sources": the forward carries each pixel's source id (the
      per-step routes composed over the whole chain) beside its value, and
      the backward is one scatter that moves the upstream gradient onto the
      marker and mask pixels those ids name.  Memory: one 32-bit id per
      pixel; nothing is recomputed and checkpoint_every is not used.  A
      forward that no backward can follow (inputs that need no gradient,
      or grad mode off) runs the plain chain instead.
  method="codes": the forward runs the chain with the fast kernels and
      keeps the state every `checkpoint_every` steps; the backward walks
      the segments from last to first, recomputes each from its checkpoint
      recording a code per pixel and step, and the reverse gather walks the
      steps back one by one.  Memory: one image per checkpoint plus one byte
      per pixel-step of a single segment.
Both give the same gradient: the same contributions, summed in another
order (float64 "codes" results equal the oracle's step-by-step scatter bit
for bit; "sources" adds with hardware atomics in no fixed order).
"""
import torch

from . import ops


def _chain(op, marker, mask, n):
    """n geodesic steps of marker under mask, all images of a batch in the
    same launches; a fresh tensor of marker's shape."""
    if n == 0:
        return marker.clone()
    imgs_m = marker if marker.dim() == 3 else marker.unsqueeze(0)
    imgs_k = mask if mask.dim() == 3 else mask.unsqueeze(0)
    return ops.geodesic_chain_batch(op, imgs_m, imgs_k, n).view_as(marker)


class GeodesicChainFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, marker, mask, n_steps, op, checkpoint_every, method, gradients_wanted=True):
        if method not in ("sources", "codes"):
            raise ValueError("method is 'sources' or 'codes'")
        if marker.dtype not in (torch.float32, torch.float64):
            raise TypeError("gradients need float32 or float64 images")
        n_steps = int(n_steps)
        seg = max(1, int(checkpoint_every))
        marker = marker.contiguous()
        mask = mask.contiguous()
        ctx.n_steps, ctx.seg, ctx.op, ctx.method = n_steps, seg, op, method
        if method == "sources":
            if not (gradients_wanted and (ctx.needs_input_grad[0] or ctx.needs_input_grad[1])):
                return _chain(op, marker, mask, n_steps)
            out, src = ops.geodesic_chain_fwd_sources(op, marker, mask, n_steps)
            ctx.save_for_backward(mask, src)
            return out
        ckpts = [marker]
        cur = marker
        starts = list(range(0, n_steps, seg))
        for i, s0 in enumerate(starts):
            cur = _chain(op, cur, mask, min(seg, n_steps - s0))
            if i + 1 < len(starts):
                ckpts.append(cur)
        # the last segment's state is a fresh tensor that no checkpoint holds
        out = cur if n_steps > 0 else marker.clone()
        ctx.save_for_backward(mask, *ckpts)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        g = grad_out.contiguous()
        if ctx.method == "sources":
            mask, src = ctx.saved_tensors
            gm = torch.zeros_like(mask)
            g = ops.geodesic_chain_bwd_sources(src, g, gm)
            return (g, gm) + (None,) * (len(ctx.needs_input_grad) - 2)
        mask, *ckpts = ctx.saved_tensors
        gm = torch.zeros_like(mask)
        starts = list(range(0, ctx.n_steps, ctx.seg))
        for i in reversed(range(len(starts))):
            n = min(ctx.seg, ctx.n_steps - starts[i])
            _, codes = ops.geodesic_chain_fwd_codes(ctx.op, ckpts[i], mask, n)
            g = ops.geodesic_chain_bwd(ctx.op, codes, g, gm)
            del codes
        # one entry per argument given to apply (gradients_wanted may be left out)
        return (g, gm) + (None,) * (len(ctx.needs_input_grad) - 2)


def geodesic_chain(marker, mask, n_steps, op="dilate", checkpoint_every=32, method="sources"):
    """Differentiable n_steps geodesic dilations ('dilate') or erosions
    ('erode') of marker under mask; (H, W) or (B, H, W) float tensors.
    method: 'sources' (source ids carried through the forward, one scatter
    back) or 'codes' (checkpoints every checkpoint_every steps, per-step
    codes and the reverse gather)."""
    # under no_grad the inputs may still require gradients; the source ids
    # are kept only when a backward can follow
    wanted = torch.is_grad_enabled() and (marker.requires_grad or mask.requires_grad)
    return GeodesicChainFunction.apply(marker, mask, n_steps, op, checkpoint_every, method, wanted)
