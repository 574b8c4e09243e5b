"""Plans, buffers and the torch.autograd.Function around libsmnn.

PyTorch only provides device memory and the current stream here.
"""
from __future__ import annotations

import ctypes
from collections import OrderedDict

import numpy as np
import torch

from . import _lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Plan:
    """A solver plan: sizes, mode and the per-level partition of a batch.

    steps: int (every instance has that many steps) or a sequence of T_i.
    init_points: T_init, the leading time points that carry the n_init
           initial values (u0 is then N x T_init x V x n_init).
    variables, equations: V coupled variables and Q governing equations
           per time point (c is S x Q x V(R+1), b is S x Q, y is S x V(R+1)).
    row_weights: w holds one weight per row (the governing weights [S][Q],
           the initial weights [N][T_init][V][n_init] and the smoothness
           weights [S], concatenated) instead of three per instance.
    mode:  'fp64' (the paper's single solve), 'fp64r' (plus row-residual
           refinement) or 'fp32r' (float32 memory traffic, float64 arithmetic,
           refinement).
    """

    def __init__(self, order: int, n_init: int, n_inst: int, steps, mode: str = "fp64r",
                 refine_steps: int = -1, chunk: int = 0, block: int = 0, max_blocks: int = 0,
                 chunk_upper: int = 0, init_points: int = 1, variables: int = 1, equations: int = 0,
                 row_weights: bool = False):
        L = _lib.lib()
        if mode not in _lib.MODES:
            raise ValueError("mode must be one of %s" % sorted(_lib.MODES))
        d = _lib.PlanDesc()
        d.order, d.n_init, d.n_inst = int(order), int(n_init), int(n_inst)
        if np.isscalar(steps):
            self._steps_arr = None
            d.steps, d.steps_uniform = None, int(steps)
            self.steps = np.full(int(n_inst), int(steps), dtype=np.int64)
        else:
            self._steps_arr = np.ascontiguousarray(steps, dtype=np.int64)
            if self._steps_arr.shape != (int(n_inst),):
                raise ValueError("steps must have one entry per instance")
            d.steps = self._steps_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            d.steps_uniform = 0
            self.steps = self._steps_arr
        d.mode, d.refine_steps, d.chunk = _lib.MODES[mode], int(refine_steps), int(chunk)
        d.chunk_upper = int(chunk_upper)
        d.block, d.max_blocks = int(block), int(max_blocks)
        d.init_points = int(init_points)
        d.variables, d.equations, d.row_weights = int(variables), int(equations), int(bool(row_weights))
        h = ctypes.c_void_p()
        _lib.check(L.smnn_plan_create(ctypes.byref(d), ctypes.byref(h)), "smnn_plan_create")
        self._h = h
        self._L = L
        self.order, self.n_init, self.n_inst, self.mode = int(order), int(n_init), int(n_inst), mode
        self.variables = int(variables)
        self.equations = int(equations) if equations else self.variables
        self.row_weights = bool(row_weights)
        self.k = self.variables * (self.order + 1)     # unknowns per time point
        self.init_points = self.query(_lib.Q_INIT_POINTS)
        fb, wb, S = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int64()
        _lib.check(L.smnn_plan_sizes(h, ctypes.byref(fb), ctypes.byref(wb), ctypes.byref(S)), "smnn_plan_sizes")
        self.factor_bytes, self.workspace_bytes, self.total_steps = fb.value, wb.value, S.value
        self.dtype = torch.float32 if mode == "fp32r" else torch.float64

    def query(self, key: int) -> int:
        return int(self._L.smnn_plan_query(self._h, key))

    @property
    def levels(self):
        n = self.query(_lib.Q_LEVELS)
        return [(self.query(1000 + l), self.query(2000 + l)) for l in range(n)]

    @property
    def chunk(self):
        return self.query(_lib.Q_CHUNK)

    @property
    def chunk_upper(self):
        return self.query(_lib.Q_CHUNK_UPPER)

    @property
    def refine_steps(self):
        return self.query(_lib.Q_REFINE)

    @property
    def top_level(self):
        """First level solved by the one-wave-per-instance launch (0: none)."""
        return self.query(_lib.Q_TOP_LEVEL)

    def trace(self, capacity: int):
        """Record a hipEvent pair around each of the next `capacity` launches."""
        _lib.check(self._L.smnn_trace_enable(self._h, int(capacity)), "smnn_trace_enable")

    def trace_read(self, cap: int = 1 << 16):
        """Traced launches since the last read (call after synchronising): a list
        of (kernel name, level, rhs form, out form, milliseconds)."""
        buf = (_lib.TraceRecord * cap)()
        n = self._L.smnn_trace_read(self._h, buf, cap)
        if n < 0:
            raise _lib.SmnnError(4, "smnn_trace_read")
        return [(_lib.KERNEL_NAMES.get(r.kernel, str(r.kernel)), r.level, r.rhs, r.out, r.ms) for r in buf[:n]]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                self._L.smnn_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    # ---------------------------------------------------------------- buffers
    def new_factor(self, device):
        return torch.empty(self.factor_bytes, dtype=torch.uint8, device=device)

    def new_workspace(self, device):
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def _check(self, name, t, shape):
        if t is None:
            raise ValueError("%s is required" % name)
        if not t.is_cuda:
            raise ValueError("%s must be a device tensor" % name)
        if t.dtype != self.dtype:
            raise TypeError("%s must be %s for mode %s" % (name, self.dtype, self.mode))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        if t.numel() != int(np.prod(shape)):
            raise ValueError("%s has %d elements, expected %s" % (name, t.numel(), shape))

    @property
    def n_initial(self):
        """Initial values per instance: T_init V n_init."""
        return self.init_points * self.variables * self.n_init

    @property
    def weight_shape(self):
        """Elements of w (and dw): (N, 3), or the per-row buffer's length."""
        if self.row_weights:
            return (self.total_steps * self.equations + self.n_inst * self.n_initial + self.total_steps,)
        return (self.n_inst, 3)

    def _check_inputs(self, c, b, h, u0, w):
        S, k, N, Q = self.total_steps, self.k, self.n_inst, self.equations
        self._check("c", c, (S, Q * k))
        self._check("b", b, (S * Q,))
        self._check("h", h, (S,))
        if self.n_init:
            self._check("u0", u0, (N, self.n_initial))
        self._check("w", w, self.weight_shape)

    def forward(self, c, b, h, u0, w, y, factor, workspace, info=None, stream=None):
        """Enqueue smnn_forward on `stream` (default: torch's current stream)."""
        self._check_inputs(c, b, h, u0, w)
        self._check("y", y, (self.total_steps, self.k))
        st = torch.cuda.current_stream(c.device).cuda_stream if stream is None else stream
        _lib.check(self._L.smnn_forward(self._h, _ptr(c), _ptr(b), _ptr(h), _ptr(u0), _ptr(w), _ptr(y),
                                        _ptr(factor), factor.numel(), _ptr(workspace), workspace.numel(),
                                        _ptr(info), ctypes.c_void_p(st)), "smnn_forward")

    def forward_noalloc(self, c, b, h, u0, w, y, factor, info=None, stream=None):
        """Enqueue smnn_forward_noalloc: smnn_forward with the library's static
        device workspace (plans whose workspace fits it; see include/smnn.h)."""
        self._check_inputs(c, b, h, u0, w)
        self._check("y", y, (self.total_steps, self.k))
        st = torch.cuda.current_stream(c.device).cuda_stream if stream is None else stream
        _lib.check(self._L.smnn_forward_noalloc(self._h, _ptr(c), _ptr(b), _ptr(h), _ptr(u0), _ptr(w), _ptr(y),
                                                _ptr(factor), factor.numel(), _ptr(info), ctypes.c_void_p(st)),
                   "smnn_forward_noalloc")

    def backward(self, c, b, h, u0, w, y, factor, gy, dc, db, dh, du0, dw, workspace, info=None, stream=None):
        """Enqueue smnn_backward on `stream` (default: torch's current stream)."""
        self._check_inputs(c, b, h, u0, w)
        S, k, N = self.total_steps, self.k, self.n_inst
        Q = self.equations
        for name, t, shape in (("y", y, (S, k)), ("gy", gy, (S, k)), ("dc", dc, (S, Q * k)), ("db", db, (S * Q,)),
                               ("dh", dh, (S,)), ("dw", dw, self.weight_shape)):
            self._check(name, t, shape)
        if self.n_init:
            self._check("du0", du0, (N, self.n_initial))
        st = torch.cuda.current_stream(c.device).cuda_stream if stream is None else stream
        _lib.check(self._L.smnn_backward(self._h, _ptr(c), _ptr(b), _ptr(h), _ptr(u0), _ptr(w), _ptr(y),
                                         _ptr(factor), factor.numel(), _ptr(gy), _ptr(dc), _ptr(db), _ptr(dh),
                                         _ptr(du0), _ptr(dw), _ptr(workspace), workspace.numel(), _ptr(info),
                                         ctypes.c_void_p(st)), "smnn_backward")


_PLANS: "OrderedDict[tuple, Plan]" = OrderedDict()


def get_plan(order, n_init, n_inst, steps, mode="fp64r", refine_steps=-1, chunk=0, init_points=1, variables=1,
             equations=0, row_weights=False):
    """Plans are cached per (device, sizes, mode); creating one uploads metadata."""
    key_steps = int(steps) if np.isscalar(steps) else tuple(int(t) for t in steps)
    key = (torch.cuda.current_device(), order, n_init, n_inst, key_steps, mode, refine_steps, chunk, init_points,
           variables, equations, bool(row_weights))
    p = _PLANS.get(key)
    if p is None:
        p = Plan(order, n_init, n_inst, steps, mode=mode, refine_steps=refine_steps, chunk=chunk,
                 init_points=init_points, variables=variables, equations=equations, row_weights=row_weights)
        _PLANS[key] = p
        while len(_PLANS) > 16:
            _PLANS.popitem(last=False)
    else:
        _PLANS.move_to_end(key)
    return p


class SmnnSolve(torch.autograd.Function):
    """y = argmin || W^{1/2} (A y - b) || (Eq. 9) with gradients from the adjoint (Eq. 14)."""

    @staticmethod
    def forward(ctx, c, b, h, u0, w, plan):
        dev = c.device
        y = torch.empty((plan.total_steps, plan.k), dtype=plan.dtype, device=dev)
        factor = plan.new_factor(dev)
        ws = plan.new_workspace(dev)
        plan.forward(c, b, h, u0, w, y, factor, ws)
        ctx.plan = plan
        ctx.save_for_backward(c, b, h, u0, w, y, factor)
        return y

    @staticmethod
    def backward(ctx, gy):
        c, b, h, u0, w, y, factor = ctx.saved_tensors
        plan = ctx.plan
        dev = c.device
        gy = gy.contiguous().to(plan.dtype)
        dc = torch.empty_like(c)
        db = torch.empty_like(b)
        dh = torch.empty_like(h)
        du0 = torch.empty_like(u0) if u0 is not None and plan.n_init else None
        dw = torch.empty_like(w)
        ws = plan.new_workspace(dev)
        plan.backward(c, b, h, u0, w, y, factor, gy, dc, db, dh, du0, dw, ws)
        return dc, db, dh, du0, dw, None


def solve(c, b, h, u0, w, order=None, n_init=None, steps=None, mode="fp64r", refine_steps=-1, chunk=0,
          variables=1, equations=0, row_weights=False, init_points=None):
    """Differentiable batched solve.

    Uniform one-variable batches may pass c as (N, T, R+1), b and h as (N, T);
    otherwise c is (S, Q V (R+1)), b is (S, Q) or (S,), h is (S,) and `steps`
    lists T_i (or is the uniform T).  u0 is (N, n_init) (initial values at the
    first point) or (N, T_init, n_init) (at each of the first T_init points)
    for one variable, (N, T_init V n_init) in general; w is (N, 3), or with
    row_weights the per-row buffer described in Plan.  Returns y with the
    shape of c (one variable) or (S, V (R+1)).
    """
    shape = c.shape
    general = variables > 1 or (equations or variables) > 1 or row_weights
    if c.dim() == 3 and not general:
        N, T, k = c.shape
        steps = T if steps is None else steps
        c2, b2, h2 = c.reshape(N * T, k), b.reshape(N * T), h.reshape(N * T)
    else:
        if steps is None or (general and (order is None or n_init is None)):
            raise ValueError("steps (and, for several variables or per-row weights, order and n_init) are required")
        N = len(steps) if not np.isscalar(steps) else (u0.shape[0] if u0 is not None else w.shape[0])
        c2, b2, h2 = c.reshape(h.numel(), -1), b.reshape(-1), h.reshape(-1)
    k = c2.shape[1] // max(1, (equations or variables))
    order = k // variables - 1 if order is None else order
    if init_points is None:
        init_points = u0.shape[1] if u0 is not None and u0.dim() == 3 and not general else 1
    if n_init is None:
        n_init = u0.shape[-1] if u0 is not None else 0
    plan = get_plan(order, n_init, N, steps, mode=mode, refine_steps=refine_steps, chunk=chunk,
                    init_points=init_points, variables=variables, equations=equations, row_weights=row_weights)
    y = SmnnSolve.apply(c2, b2, h2, u0, w, plan)
    return y.reshape(shape) if not general else y
