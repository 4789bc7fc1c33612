"""Differentiable geodesic chains with activation checkpointing.

GeodesicChainFunction: forward runs the chain with the fast kernels and
keeps the state every `checkpoint_every` steps; backward walks the segments
from last to first and recomputes each one from its checkpoint, then takes
the gradient through it in one of two ways:
  method="sources": the recomputation carries each pixel's source id (the
      per-step routes composed over the segment), and one scatter moves
      the segment's upstream gradient onto the marker and mask pixels;
      memory: one image per checkpoint plus one 32-bit id per pixel;
  method="codes": the recomputation records a code per pixel and step, and
      the reverse gather walks the steps back one by one; memory: one image
      per checkpoint plus one byte per pixel-step of a single segment.
Both give the same gradient: the same contributions, summed in another
order (float64 "codes" results equal the oracle's step-by-step scatter bit
for bit; "sources" adds with hardware atomics in no fixed order).
"""
import torch

from . import ops


class GeodesicChainFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, marker, mask, n_steps, op, checkpoint_every, method):
        if method not in ("sources", "codes"):
            raise ValueError("method is 'sources' or 'codes'")
        if marker.dtype not in (torch.float32, torch.float64):
            raise TypeError("gradients need float32 or float64 images")
        n_steps = int(n_steps)
        seg = max(1, int(checkpoint_every))
        marker = marker.contiguous()
        mask = mask.contiguous()
        imgs_m = marker if marker.dim() == 3 else marker.unsqueeze(0)
        imgs_k = mask if mask.dim() == 3 else mask.unsqueeze(0)
        ckpts = [marker]
        cur = imgs_m
        starts = list(range(0, n_steps, seg))
        for i, s0 in enumerate(starts):
            n = min(seg, n_steps - s0)
            # all images of the batch in the same launches
            cur = ops.geodesic_chain_batch(op, cur, imgs_k, n)
            if i + 1 < len(starts):
                ckpts.append(cur.view_as(marker))
        # the last segment's state is a fresh tensor that no checkpoint holds
        out = cur.view_as(marker) if n_steps > 0 else marker.clone()
        ctx.n_steps, ctx.seg, ctx.op, ctx.method = n_steps, seg, op, method
        ctx.save_for_backward(mask, *ckpts)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        mask, *ckpts = ctx.saved_tensors
        g = grad_out.contiguous()
        gm = torch.zeros_like(mask)
        starts = list(range(0, ctx.n_steps, ctx.seg))
        for i in reversed(range(len(starts))):
            n = min(ctx.seg, ctx.n_steps - starts[i])
            if ctx.method == "sources":
                _, src = ops.geodesic_chain_fwd_sources(ctx.op, ckpts[i], mask, n)
                g = ops.geodesic_chain_bwd_sources(src, g, gm)
                del src
            else:
                _, codes = ops.geodesic_chain_fwd_codes(ctx.op, ckpts[i], mask, n)
                g = ops.geodesic_chain_bwd(ctx.op, codes, g, gm)
                del codes
        return g, gm, None, None, None, None


def geodesic_chain(marker, mask, n_steps, op="dilate", checkpoint_every=32, method="sources"):
    """Differentiable n_steps geodesic dilations ('dilate') or erosions
    ('erode') of marker under mask; (H, W) or (B, H, W) float tensors.
    method: 'sources' (composed routes, one scatter per segment) or 'codes'
    (per-step codes and reverse gather)."""
    return GeodesicChainFunction.apply(marker, mask, n_steps, op, checkpoint_every, method)
