"""Early-exit gaze network (Sec. 3.2), for its latency on the host CPU.

A vision transformer over the eye image: a convolutional patch embedding, a
class token and learned positions, 6 blocks of 6-head self-attention with
embedding size 384 and an MLP, and after every block a linear exit that maps
the class token to a 2D gaze.  Optional tokenwise pruning after each block
drops the patch tokens the class token attends to least (a fraction per
block; the paper thresholds the attention score).

The paper trains it on eye images that are not available here, so the
weights are random (seeded): the predictions carry no information and the
module is used for what it costs -- the per-exit latency of the tracker that
runs beside the renderer (Algorithm 1) -- on the CPU, where the method puts
it.  Plain PyTorch CPU operations.
"""
from __future__ import annotations

import math
import time

import torch
from torch import nn


class Block(nn.Module):
    def __init__(self, dim, heads, mlp_ratio=4):
        super().__init__()
        self.heads = heads
        self.n1 = nn.LayerNorm(dim)
        self.qkv = nn.Linear(dim, 3 * dim)
        self.proj = nn.Linear(dim, dim)
        self.n2 = nn.LayerNorm(dim)
        self.mlp = nn.Sequential(nn.Linear(dim, mlp_ratio * dim), nn.GELU(), nn.Linear(mlp_ratio * dim, dim))

    def forward(self, x):
        """x [B][T][D] -> (x, attention of the class token to every token, averaged over heads [B][T])."""
        B, T, D = x.shape
        h = self.heads
        q, k, v = self.qkv(self.n1(x)).reshape(B, T, 3, h, D // h).permute(2, 0, 3, 1, 4)
        att = torch.softmax((q @ k.transpose(-2, -1)) / math.sqrt(D // h), dim=-1)  # [B][h][T][T]
        y = (att @ v).transpose(1, 2).reshape(B, T, D)
        x = x + self.proj(y)
        x = x + self.mlp(self.n2(x))
        return x, att[:, :, 0, :].mean(dim=1)


class EarlyExitViT(nn.Module):
    def __init__(self, img=(400, 640), patch=16, dim=384, depth=6, heads=6, prune=0.0, seed=0):
        super().__init__()
        g = torch.Generator().manual_seed(seed)
        self.embed = nn.Conv2d(1, dim, patch, stride=patch)
        n_tok = (img[0] // patch) * (img[1] // patch)
        self.cls = nn.Parameter(torch.zeros(1, 1, dim))
        self.pos = nn.Parameter(torch.zeros(1, n_tok + 1, dim))
        self.blocks = nn.ModuleList([Block(dim, heads) for _ in range(depth)])
        self.exits = nn.ModuleList([nn.Linear(dim, 2) for _ in range(depth)])
        self.prune = float(prune)
        with torch.no_grad():
            for p in self.parameters():
                p.copy_(torch.randn(p.shape, generator=g) * 0.02)

    @torch.no_grad()
    def exits_iter(self, img):
        """Yields (exit index 1..depth, gaze [B][2]) as each block finishes."""
        x = self.embed(img).flatten(2).transpose(1, 2)
        x = torch.cat([self.cls.expand(x.shape[0], -1, -1), x], dim=1) + self.pos
        for i, (blk, head) in enumerate(zip(self.blocks, self.exits)):
            x, cls_att = blk(x)
            yield i + 1, head(x[:, 0])
            if self.prune > 0.0 and i + 1 < len(self.blocks):
                keep = max(1, int(round((x.shape[1] - 1) * (1.0 - self.prune))))
                idx = cls_att[:, 1:].topk(keep, dim=1).indices.sort(dim=1).values + 1
                x = torch.cat([x[:, :1], torch.gather(x, 1, idx[..., None].expand(-1, -1, x.shape[2]))], dim=1)


def exit_latencies(model, img, reps=3):
    """Cumulative wall time (ms) at which each exit's prediction is out, median of reps."""
    runs = []
    for _ in range(reps):
        t0 = time.perf_counter()
        runs.append([(time.perf_counter() - t0) * 1000.0 for _ in model.exits_iter(img)])
    return [sorted(r[k] for r in runs)[len(runs) // 2] for k in range(len(runs[0]))]
