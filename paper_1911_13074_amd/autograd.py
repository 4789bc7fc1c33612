"""Differentiable geodesic chains with activation checkpointing.

GeodesicChainFunction: forward runs the chain with the fast kernels and
keeps the state every `checkpoint_every` steps; backward walks the segments
from last to first, recomputes each one from its checkpoint with the
code-recording kernel and runs the reverse gather over it.  Memory: one
image per checkpoint plus one byte per pixel-step of a single segment.
"""
import torch

from . import ops


class GeodesicChainFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, marker, mask, n_steps, op, checkpoint_every):
        if marker.dtype not in (torch.float32, torch.float64):
            raise TypeError("gradients need float32 or float64 images")
        n_steps = int(n_steps)
        seg = max(1, int(checkpoint_every))
        marker = marker.contiguous()
        mask = mask.contiguous()
        imgs_m = marker if marker.dim() == 3 else marker.unsqueeze(0)
        imgs_k = mask if mask.dim() == 3 else mask.unsqueeze(0)
        chain = ops.geodesic_dilate_chain if op == "dilate" else ops.geodesic_erode_chain
        ckpts = [marker]
        cur = imgs_m
        starts = list(range(0, n_steps, seg))
        for i, s0 in enumerate(starts):
            n = min(seg, n_steps - s0)
            nxt = torch.empty_like(cur)
            for b in range(cur.shape[0]):
                chain(cur[b], imgs_k[b], n, out=nxt[b])
            cur = nxt
            if i + 1 < len(starts):
                ckpts.append(cur.view_as(marker))
        # the last segment's state is a fresh tensor that no checkpoint holds
        out = cur.view_as(marker) if n_steps > 0 else marker.clone()
        ctx.n_steps, ctx.seg, ctx.op = n_steps, seg, op
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
            _, codes = ops.geodesic_chain_fwd_codes(ctx.op, ckpts[i], mask, n)
            g = ops.geodesic_chain_bwd(ctx.op, codes, g, gm)
            del codes
        return g, gm, None, None, None


def geodesic_chain(marker, mask, n_steps, op="dilate", checkpoint_every=32):
    """Differentiable n_steps geodesic dilations ('dilate') or erosions
    ('erode') of marker under mask; (H, W) or (B, H, W) float tensors."""
    return GeodesicChainFunction.apply(marker, mask, n_steps, op, checkpoint_every)
