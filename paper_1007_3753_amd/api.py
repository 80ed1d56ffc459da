"""Thin Python binding over the libl1alm C ABI.

Only argument marshalling happens here: tensors are laid out column-major
(one instance per column) and their device pointers, sizes and the current
HIP stream are handed to the library, which runs every step of the method.
PyTorch provides device memory and streams.
"""
import ctypes
import sys

import torch

from . import _lib

PROBLEMS = {"p1": 0, "p12": 1, "qp": 2}
STRUCTURES = {"dense": 0, "cab": 1}
METHODS = {"dalm": 0, "palm": 1, "dalm_cg1": 2}
PRECISIONS = {"fp32": 0, "bf16_refine": 1, "bf16x3": 2}
FORMS = {"auto": 0, "dense": 1, "structured": 2}
CONVERGED, MAXITER, NONFINITE, DIVERGED = 0, 1, 2, 3


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _colmajor(t, rows):
    """(rows, N) tensor -> contiguous float32 (N, rows) buffer = column-major (rows x N)."""
    t = torch.as_tensor(t)
    if t.dim() == 1:
        t = t[:, None]
    if t.shape[0] != rows:
        raise ValueError(f"expected {rows} rows, got shape {tuple(t.shape)}")
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU")
    return t.t().contiguous().to(torch.float32)


class SolveResult:
    def __init__(self, x, e, y, iters, status):
        self.x, self.e, self.y, self.iters, self.status = x, e, y, iters, status

    def __iter__(self):
        return iter((self.x, self.e, self.y, self.iters, self.status))


class Plan:
    """A factorised dictionary ready for batched solves.

    ``A`` is the (m, n_dict) dictionary on the GPU (B for ``structure="cab"``,
    where the solver works on [B, I]).  See include/l1_alm.h for the options.
    """

    def __init__(self, A, *, problem="p1", structure="dense", method="dalm",
                 precision="fp32", max_batch=1, lam=0.0, beta=0.0, xi=0.0, xi_growth=1.0,
                 max_inner=100, tol_inner=0.0, refine_switch=0.0, record_tape=False,
                 checkpoint_every=10, time_kernels=False, div_factor=0.0, iteration_form="auto"):
        self.lib = _lib.load()
        A = torch.as_tensor(A)
        if A.dim() != 2 or not A.is_cuda:
            raise ValueError("A must be a 2-D GPU tensor")
        self.m, self.n_dict = int(A.shape[0]), int(A.shape[1])
        self.problem, self.structure, self.method = problem, structure, method
        self.precision = precision
        self.max_batch = int(max_batch)
        self.split = structure == "cab" or problem == "p12"
        self.n_full = self.n_dict + (self.m if self.split else 0)
        self.device = A.device
        Ac = A.t().contiguous().to(torch.float32)   # column-major m x n_dict
        d = _lib.l1_alm_desc()
        d.m, d.n_dict, d.lda = self.m, self.n_dict, self.m
        d.problem, d.structure = PROBLEMS[problem], STRUCTURES[structure]
        d.method, d.precision = METHODS[method], PRECISIONS[precision]
        d.max_batch = self.max_batch
        d.lam, d.beta, d.xi, d.xi_growth = float(lam), float(beta), float(xi), float(xi_growth)
        d.max_inner, d.tol_inner, d.refine_switch = int(max_inner), float(tol_inner), float(refine_switch)
        d.record_tape, d.checkpoint_every = int(bool(record_tape)), int(checkpoint_every)
        d.time_kernels = int(bool(time_kernels))
        d.div_factor = float(div_factor)
        d.iteration_form = FORMS[iteration_form]
        self.desc = d
        self._tape_N = 0
        h = ctypes.c_void_p()
        if Ac.numel() == 0:
            Ac = torch.zeros(1, device=A.device)
        _lib.check(self.lib.l1_alm_plan(ctypes.byref(d), _ptr(Ac), _stream(), ctypes.byref(h)))
        self.handle = h
        _lib.register(self)

    def close(self):
        """Release the plan's device memory (idempotent)."""
        if getattr(self, "handle", None):
            self.lib.l1_alm_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        # at interpreter shutdown the atexit hook of _lib has closed the plan
        # already; never call into the library from a finalizing interpreter
        if sys is None or sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def solve(self, b, *, tol=1e-6, max_iter=10000, eps=None, w0=None, y0=None,
              want_y=True, pen=None):
        """Solve the columns of ``b`` (m, N).  Returns SolveResult with
        x (n_dict, N), e (m, N) or None, y (m, N) or None, iters (N,), status (N,).
        ``max_iter < 0`` runs exactly ``-max_iter`` iterations.  ``pen``: N
        per-instance penalties (DALM beta / PALM xi) held constant for the
        solve, or None for the plan's setting."""
        bc = _colmajor(b, self.m)
        N = bc.shape[0]
        dev = bc.device
        x = torch.empty(N, self.n_dict, device=dev, dtype=torch.float32)
        has_e = self.split or (self.method == "palm" and self.problem == "qp")
        e = torch.empty(N, self.m, device=dev, dtype=torch.float32) if has_e else None
        y = torch.empty(N, self.m, device=dev, dtype=torch.float32) if (want_y and self.method in ("dalm", "dalm_cg1")) else None
        iters = torch.empty(N, device=dev, dtype=torch.int32)
        status = torch.empty(N, device=dev, dtype=torch.int32)
        epsc = None
        if eps is not None:
            epsc = torch.as_tensor(eps, dtype=torch.float32, device=dev).reshape(-1).contiguous()
            if epsc.numel() == 1 and N > 1:
                epsc = epsc.expand(N).contiguous()
        penc = None
        if pen is not None:
            penc = torch.as_tensor(pen, dtype=torch.float32, device=dev).reshape(-1).contiguous()
            if penc.numel() == 1 and N > 1:
                penc = penc.expand(N).contiguous()
            if penc.numel() != N:
                raise ValueError(f"pen must hold {N} values")
        w0c = _colmajor(w0, self.n_full) if w0 is not None else None
        y0c = _colmajor(y0, self.m) if y0 is not None else None
        _lib.check(self.lib.l1_alm_solve(
            self.handle, _ptr(bc), self.m, N, _ptr(epsc), _ptr(penc), ctypes.c_float(tol), int(max_iter),
            _ptr(w0c), _ptr(y0c), _ptr(x), max(self.n_dict, 1), _ptr(e), self.m, _ptr(y), self.m,
            _ptr(iters), _ptr(status), _stream()))
        if max_iter < 0 and self.desc.record_tape:
            self._tape_N = N
        return SolveResult(x.t(), None if e is None else e.t(), None if y is None else y.t(),
                           iters, status)

    def set_ksplit(self, table):
        """Install a split-K table (parts by active 64-instance column tiles
        1..len(table); 0 keeps the heuristic); an empty table clears it."""
        t = (ctypes.c_int * max(len(table), 1))(*[int(v) for v in table])
        _lib.check(self.lib.l1_alm_set_ksplit(self.handle, t, len(table)))

    def tune_ksplit(self, iters=256):
        """Run the split-K autotuner of l1_alm_tune_ksplit on this plan and
        return the table it installed (8 entries)."""
        out = (ctypes.c_int * 8)()
        _lib.check(self.lib.l1_alm_tune_ksplit(self.handle, int(iters), out, 8, _stream()))
        return list(out)

    def backward(self, gx, ge=None):
        """Reverse-mode product of the last recorded fixed-count solve: given
        the adjoints of its outputs x (n_dict, N) and e (m, N), returns
        (gb (m, N), gA (m, n_dict)) = gradients with respect to b and the
        dictionary."""
        gxc = _colmajor(gx, self.n_dict)
        N = self._tape_N or gxc.shape[0]
        gec = _colmajor(ge, self.m) if (ge is not None and self.split) else None
        if gxc.shape[0] != N or (gec is not None and gec.shape[0] != N):
            raise ValueError("adjoints must have one column per recorded instance")
        gb = torch.empty(N, self.m, device=gxc.device, dtype=torch.float32)
        gA = torch.zeros(self.n_dict, self.m, device=gxc.device, dtype=torch.float32)
        _lib.check(self.lib.l1_alm_backward(self.handle, _ptr(gxc), _ptr(gec), _ptr(gb), _ptr(gA),
                                            _stream()))
        return gb.t(), gA.t()

    def kkt(self, b, x, e=None, y=None, eps=None):
        """FP64 certificate per instance: (N, 4) float64 tensor of
        [primal residual, dual infeasibility, sign disagreement, gap]."""
        bc = _colmajor(b, self.m)
        N = bc.shape[0]
        xc = _colmajor(x, self.n_dict)
        ec = _colmajor(e, self.m) if e is not None else None
        yc = _colmajor(y, self.m) if y is not None else None
        epsc = None if eps is None else torch.as_tensor(eps, dtype=torch.float32, device=bc.device).reshape(-1).contiguous()
        rep = torch.empty(N, 4, device=bc.device, dtype=torch.float64)
        _lib.check(self.lib.l1_alm_kkt(self.handle, _ptr(bc), self.m, N, _ptr(epsc), _ptr(xc),
                                       max(self.n_dict, 1), _ptr(ec), self.m, _ptr(yc), self.m,
                                       _ptr(rep), _stream()))
        return rep

    STAT_KEYS = ("launch_fp32", "launch_bf16", "launch_split", "cols_fp32", "cols_bf16",
                 "cols_split", "timed_ms", "timed_launches", "iterations", "solve_ms", "plan_ms",
                 "inner_iterations", "cols_structured")

    def last_stats(self):
        out = (ctypes.c_double * 14)()
        _lib.check(self.lib.l1_alm_last_stats(self.handle, out, 14))
        return dict(zip(self.STAT_KEYS, list(out)))


def classify(x, class_ptr):
    """The recognition criterion of the face experiments (Sec. VI-B) on the
    GPU: ``x`` (n_dict, N) representations, ``class_ptr`` (C + 1,) column
    ranges of the subjects.  Returns (mass (C, N), label (N,), score (N,))
    from l1_alm_classify."""
    lib = _lib.load()
    x = torch.as_tensor(x)
    if x.dim() == 1:
        x = x[:, None]
    xc = _colmajor(x, x.shape[0])
    N, n_dict = int(xc.shape[0]), int(xc.shape[1])
    ptr = torch.as_tensor(class_ptr, dtype=torch.int32, device=xc.device).contiguous()
    C = int(ptr.numel()) - 1
    mass = torch.empty(N, C, device=xc.device, dtype=torch.float32)
    label = torch.empty(N, device=xc.device, dtype=torch.int32)
    score = torch.empty(N, device=xc.device, dtype=torch.float32)
    _lib.check(lib.l1_alm_classify(_ptr(xc), n_dict, n_dict, N, _ptr(ptr), C, _ptr(mass),
                                   _ptr(label), _ptr(score), _stream()))
    return mass.t(), label, score


def class_residuals(A, x, b, class_ptr, e=None):
    """The residual rule of the sparse-representation classifier (Sec. I,
    Sec. II-A) on the GPU: ``A`` (m, n_dict) the dictionary, ``x``
    (n_dict, N), ``b`` (m, N), ``e`` (m, N) or None, ``class_ptr`` (C + 1,).
    Returns (res (C, N), label (N,)) from l1_alm_class_residuals."""
    lib = _lib.load()
    A = torch.as_tensor(A)
    m, n_dict = int(A.shape[0]), int(A.shape[1])
    Ac = _colmajor(A, m)
    xc = _colmajor(x, n_dict)
    bc = _colmajor(b, m)
    N = int(xc.shape[0])
    ec = None if e is None else _colmajor(e, m)
    ptr = torch.as_tensor(class_ptr, dtype=torch.int32, device=xc.device).contiguous()
    C = int(ptr.numel()) - 1
    res = torch.empty(N, C, device=xc.device, dtype=torch.float32)
    label = torch.empty(N, device=xc.device, dtype=torch.int32)
    _lib.check(lib.l1_alm_class_residuals(_ptr(Ac), m, n_dict, m, _ptr(xc), n_dict,
                                          None if ec is None else _ptr(ec), m, _ptr(bc), m, N, _ptr(ptr), C,
                                          _ptr(res), _ptr(label), _stream()))
    return res.t(), label


def align(B, b, tol=1e-3, max_iter=1000, fixed_iters=None):
    """The l1 problem of the alignment step (Sec. II-B; Sec. VI-C) on the
    GPU: ``B`` (N, m, k) per-instance dictionaries, ``b`` (m, N).  Runs the
    primal ALM of l1_alm_align until ||w_new - w|| < tol ||w|| (at most
    ``max_iter`` iterations), or exactly ``fixed_iters`` iterations.
    Returns (w (k, N), e (m, N), iters (N,), status (N,)).  The library
    reads each B_j and b column-major: ``B`` given as ``Bt.transpose(1, 2)``
    of a contiguous (N, k, m) float32 tensor and ``b`` as ``bt.t()`` of a
    contiguous (N, m) one are passed without a copy."""
    lib = _lib.load()
    B = torch.as_tensor(B)
    b = torch.as_tensor(b)
    if b.dim() == 1:
        b = b[:, None]
    if B.dim() == 2:
        B = B[None]
    N, m, k = (int(v) for v in B.shape)
    if b.shape != (m, N):
        raise ValueError(f"b must be ({m}, {N}), got {tuple(b.shape)}")
    if not B.is_cuda:
        raise ValueError("tensors must live on the GPU")
    # each B_j column-major: (N, k, m) row-major holds B_j^T contiguously
    Bc = B.to(torch.float32).transpose(1, 2).contiguous()
    bc = _colmajor(b, m)
    w = torch.empty(N, k, device=bc.device, dtype=torch.float32)
    e = torch.empty(N, m, device=bc.device, dtype=torch.float32)
    iters = torch.empty(N, device=bc.device, dtype=torch.int32)
    status = torch.empty(N, device=bc.device, dtype=torch.int32)
    cap = -int(fixed_iters) if fixed_iters is not None else int(max_iter)
    _lib.check(lib.l1_alm_align(_ptr(Bc), m, k, N, _ptr(bc), m, float(tol), cap, _ptr(w), _ptr(e), m,
                                _ptr(iters), _ptr(status), _stream()))
    return w.t(), e.t(), iters, status


class DALMUnrolled(torch.autograd.Function):
    """``x, e = DALMUnrolled.apply(b, B, beta, iters, checkpoint_every)``:
    exactly ``iters`` dual ALM iterations (Algorithm 2) on the
    cross-and-bouquet matrix [B, I] from w = 0, y = 0, as a differentiable
    map of b (m, N) and B (m, n_B) with the penalty ``beta`` (N values, or
    one for all) an input held constant: the gradients are those of the map
    at fixed beta (beta itself gets none).  The forward solve and the
    backward pass both run in the library (the backward recomputes the
    iterations from checkpoints kept every ``checkpoint_every``
    iterations)."""

    @staticmethod
    def forward(ctx, b, B, beta, iters=50, checkpoint_every=10):
        b = b.detach()
        B = B.detach()
        beta = torch.as_tensor(beta, dtype=torch.float32, device=b.device).detach().reshape(-1)
        if beta.numel() == 1:
            beta = beta.expand(b.shape[1])
        if beta.numel() != b.shape[1] or not bool(torch.all(beta > 0)):
            raise ValueError("beta must hold one positive value per column of b (or one for all)")
        plan = Plan(B, structure="cab", precision="fp32", max_batch=b.shape[1],
                    record_tape=True, checkpoint_every=int(checkpoint_every))
        r = plan.solve(b, max_iter=-int(iters), want_y=False, pen=beta)
        ctx.plan = plan
        return r.x, r.e

    @staticmethod
    def backward(ctx, gx, ge):
        plan = ctx.plan
        if gx is None:
            gx = torch.zeros(plan.n_dict, plan.max_batch, device=plan.device)
        if ge is None:
            ge = torch.zeros(plan.m, plan.max_batch, device=plan.device)
        gb, gB = plan.backward(gx, ge)
        ctx.plan = None
        plan.close()
        return gb, gB, None, None, None
