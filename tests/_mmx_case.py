"""Helpers shared by the GPU tests: build a libmmx context and the matching
oracle problem from one description, move arrays to and from the device."""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from oracle import Grid, Material

BIT = {"exchange": 1, "dmi": 2, "anisotropy": 4, "zeeman": 8, "demag": 16, "thermal": 32}


@dataclass
class Case:
    n: tuple
    cell: tuple
    pbc: tuple = (0, 0, 0)
    images: tuple = (0, 0, 0)
    R: int = 1
    Ms: float = 8e5
    A: float = 1.3e-11
    alpha: float = 0.3
    Ku: float = 0.0
    u: tuple = (0.0, 0.0, 1.0)
    D: float = 0.0
    B: tuple = (0.0, 0.0, 0.0)
    T: float = 0.0
    seeds: list = field(default_factory=list)
    terms: tuple = ("exchange", "dmi", "anisotropy", "zeeman", "demag")

    @property
    def grid(self):
        return Grid(tuple(self.n), tuple(self.cell), tuple(self.pbc), tuple(self.images))

    def material(self, only=None):
        """Oracle material with the same enabled terms (``only`` restricts)."""
        t = self.terms if only is None else only
        return Material(Ms=self.Ms, A=self.A if "exchange" in t or "dmi" in t else 0.0,
                        alpha=self.alpha,
                        Ku=self.Ku if "anisotropy" in t else 0.0, u=self.u,
                        D=self.D if "dmi" in t else 0.0,
                        B=self.B if "zeeman" in t else (0.0, 0.0, 0.0),
                        T=self.T if "thermal" in t else 0.0,
                        demag="demag" in t)

    def mask(self, only=None):
        t = self.terms if only is None else only
        return sum(BIT[k] for k in t)


def open_ctx(case: Case, prec, groups=None):
    """Create, configure and return a context for ``case`` (or several cases
    as groups)."""
    import torch
    import paper_2608_15253_amd as mmx
    cases = groups if groups is not None else [case]
    grps = [mmx.make_group(c.n, c.cell, c.pbc, c.images, c.R) for c in cases]
    ctx = mmx.mmx_create(grps, prec)
    mmx.mmx_set_stream(ctx, torch.cuda.current_stream().cuda_stream)
    for g, c in enumerate(cases):
        mmx.mmx_set_material(ctx, g, c.Ms, c.A, c.alpha, c.Ku, c.u, c.D)
        mmx.mmx_set_field(ctx, g, c.B)
        if c.seeds:
            mmx.mmx_set_thermal(ctx, g, [c.T] * c.R, c.seeds)
    mmx.mmx_set_terms(ctx, case.mask())
    if "demag" in case.terms:
        mmx.mmx_build_demag(ctx)
    return ctx


def dev(a, prec):
    import torch
    import paper_2608_15253_amd as mmx
    dt = torch.float64 if prec == mmx.MMX_F64 else torch.float32
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0").contiguous()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.double().cpu().numpy()
