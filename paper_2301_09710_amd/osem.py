"""Ordered-subsets EM on libspect (the OSEM reconstructions the paper
compares against, Sec. III-A).

A subset of views is a plan of its own: its explicit view angles and its
slice of the PSFs, so the kernels need no subset logic.  Subset s holds the
views l with l mod nsub = s (the usual interleaving; the paper does not say
how its subsets are formed).  One OSEM iteration runs one ML-EM update per
subset, in order, each with the subset's own sensitivity image.
"""
from __future__ import annotations

import math

from . import spect

__all__ = ["OSEM", "subsets"]


def subsets(nview: int, nsub: int):
    return [list(range(s, nview, nsub)) for s in range(nsub)]


class OSEM:
    def __init__(self, mu, psf, dy, nsub: int, angles=None, cache_mubar=False, precision="fp32"):
        import torch
        nview = psf.shape[0]
        if not 1 <= nsub <= nview:
            raise ValueError("need 1 <= nsub <= nview")
        if angles is None:
            angles = [2.0 * math.pi * l / nview for l in range(nview)]
        self.nview, self.nsub = nview, nsub
        self.subs = subsets(nview, nsub)
        self.plans = []
        self._psf = []
        for views in self.subs:
            idx = torch.tensor(views, device=psf.device)
            p = psf.index_select(0, idx).contiguous()
            self._psf.append(p)                      # the plan borrows it
            self.plans.append(spect.Plan(mu, p, dy, angles=[angles[l] for l in views],
                                         cache_mubar=cache_mubar, precision=precision))
        self._sens = None

    def _split(self, v):
        import torch
        return [v.index_select(0, torch.tensor(s, device=v.device)).contiguous() for s in self.subs]

    def sensitivities(self):
        import torch
        if self._sens is None:
            self._sens = [p.back(torch.ones(p.proj_shape, dtype=torch.float32, device=p.device))
                          for p in self.plans]
        return self._sens

    def run(self, x, y, r=None, iters=1):
        """``iters`` OSEM iterations in place on x from the full sinogram y
        ([nview][nz][nx]) and background r (or None)."""
        ys = self._split(y)
        rs = self._split(r) if r is not None else [None] * self.nsub
        sens = self.sensitivities()
        for _ in range(iters):
            for p, ys_, rs_, s in zip(self.plans, ys, rs, sens):
                p.em_step(x, ys_, s, rs_)
        return x

    def close(self):
        for p in self.plans:
            p.close()
