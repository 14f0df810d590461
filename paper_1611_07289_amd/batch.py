"""Several independent reconstructions in one plan, with the SR iteration
captured once in a HIP graph by the library (pvr_sr_graph_create) and
replayed.

All problems of the plan share every launch (one simulate, one set of EM
kernels with one workgroup per problem for the per-problem statistics, one
gather, one update), so a graph replay of two SR iterations (ping-pong
volumes) issues the whole batch's work without host involvement.  The first
iteration after a build runs eagerly: it starts EM (sigma^2, c) for the cycle
and prepares the adjoint's brick index, which needs one host synchronisation
and therefore cannot be captured.
"""
from __future__ import annotations

from typing import Optional

from . import pvr


class GraphedSR:
    def __init__(self, plan, y, X, params: Optional[pvr.SRParams] = None):
        import torch
        self.plan, self.y = plan, y
        self.prm = params or pvr.SRParams.make()
        dev = y.device
        f32 = dict(dtype=torch.float32, device=dev)
        self.X = X
        self.Xn = torch.empty(plan.V, **f32)
        self.e = torch.empty(plan.N, **f32)
        self.p = torch.empty(plan.N, **f32)
        self.pbar = torch.empty(plan.M, **f32)
        self.W = torch.empty(plan.M, **f32)
        self.num = torch.empty(plan.V, **f32)
        self.den = torch.empty(plan.V, **f32)
        self.em = plan.em_state(dev)
        self.graph = None

    def _iter(self, src, dst, flags=0):
        pl = self.plan
        pl.simulate(src, y_obs=self.y, resid=self.e)
        pl.robust_weights(self.e, self.y, self.em, self.p, self.pbar, self.W,
                          flags | pvr.PVR_EM_RESID_FRESH | pvr.PVR_EM_PREP_ADJOINT)
        pl.backproject(self.e, self.p, self.W, self.num, self.den)
        pl.sr_update(src, self.num, self.den, dst, self.prm)

    def start(self):
        """Eager first iteration of a cycle (EM start), result back in X."""
        self._iter(self.X, self.Xn, pvr.PVR_EM_INIT)
        self.X.copy_(self.Xn)

    def capture(self):
        """Two SR iterations (X -> Xn -> X) recorded in one graph."""
        if self.graph is not None:
            self.graph.close()
        self.graph = pvr.SRGraph(self.plan, self.X, self.Xn, self.y, self.e, self.p, self.pbar,
                                 self.W, self.num, self.den, self.em, self.prm, iters=2)
        return self.graph

    def replay_pairs(self, n_pairs: int):
        """2 * n_pairs SR iterations; the volume ends in X."""
        for _ in range(n_pairs):
            self.graph.launch()
