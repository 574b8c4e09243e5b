"""Capture of one forward (+ backward) solve into a HIP graph.

The library's forward and backward calls allocate nothing, read nothing back
and clear their scratch with kernels, so torch's graph capture records them
as plain kernel nodes; replay() re-runs the whole multi-level launch
sequence with one submission.  Buffers are fixed at capture time: write new
inputs into c, b, h, u0, w, gy in place and replay.
"""
from __future__ import annotations

import torch


class CapturedSolve:
    def __init__(self, plan, c, b, h, u0, w, y, factor, workspace, gy=None, grads=None):
        self.plan = plan
        args_f = (c, b, h, u0, w, y, factor, workspace)
        args_b = None
        if gy is not None:
            dc, db, dh, du0, dw = grads
            args_b = (c, b, h, u0, w, y, factor, gy, dc, db, dh, du0, dw, workspace)

        def run():
            plan.forward(*args_f)
            if args_b is not None:
                plan.backward(*args_b)

        # warm up on a side stream (default priority), as graph capture requires
        side = torch.cuda.Stream(device=c.device)
        side.wait_stream(torch.cuda.current_stream(c.device))
        with torch.cuda.stream(side):
            run()
        torch.cuda.current_stream(c.device).wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            run()

    def replay(self):
        self.graph.replay()
