"""Torch-facing wrappers over the C ABI.  Tensors supply device memory and the
stream; every computation runs in the HIP library.

Builders are (S, N, N) complex128 or complex64 CUDA tensors; gates are
(..., 4, 4) complex128; locations are (p, 2) integer arrays (host)."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _native as nat

_CTX: dict[int, ctypes.c_void_p] = {}


def _dev_index(device) -> int:
    if device is None:
        return torch.cuda.current_device()
    if isinstance(device, int):
        return device
    d = torch.device(device)
    return d.index if d.index is not None else torch.cuda.current_device()


def _ctx(device: torch.device | int | None = None) -> ctypes.c_void_p:
    """Library context for the device, bound to torch's current stream."""
    lib = nat.load()
    dev = _dev_index(device)
    ctx = _CTX.get(dev)
    if ctx is None:
        ctx = ctypes.c_void_p()
        nat.check(lib.qf_create(ctypes.byref(ctx), dev, None))
        _CTX[dev] = ctx
    stream = torch.cuda.current_stream(dev).cuda_stream
    nat.check(lib.qf_set_stream(ctx, ctypes.c_void_p(stream)), ctx)
    return ctx


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _loc(loc) -> ctypes.Array:
    a = np.ascontiguousarray(np.asarray(loc, dtype=np.int32).reshape(-1))
    return (ctypes.c_int32 * a.size)(*a.tolist())


def _prec(t: torch.Tensor) -> int:
    if t.dtype == torch.complex128:
        return nat.QF_C128
    if t.dtype == torch.complex64:
        return nat.QF_C64
    raise TypeError(f"builder dtype must be complex128 or complex64, got {t.dtype}")


def _n_of(N: int) -> int:
    n = N.bit_length() - 1
    if 1 << n != N:
        raise ValueError(f"matrix size {N} is not a power of two")
    return n


def _check_builder(b: torch.Tensor) -> tuple[int, int]:
    if not b.is_cuda or not b.is_contiguous() or b.dim() != 3 or b.shape[1] != b.shape[2]:
        raise ValueError("builder must be a contiguous CUDA tensor of shape (S, N, N)")
    return b.shape[0], _n_of(b.shape[1])


def _c128(t: torch.Tensor, shape) -> torch.Tensor:
    if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected a contiguous CUDA complex128 tensor of shape {tuple(shape)}, got "
                         f"{t.dtype} {tuple(t.shape)}")
    return t


def set_pass_tile(device, precision: int, n: int, gate_class: int, tile: int) -> None:
    """Fix the pass form for (precision, n, gate class): -1 register-direct,
    -2 micro-tile (complex64), 256/512/1024 LDS tile columns, 0 = tune again
    (qf_set_pass_tile)."""
    ctx = _ctx(device)
    nat.check(nat.load().qf_set_pass_tile(ctx, precision, n, gate_class, tile), ctx)


def set_pass2_tiles(device, precision: int, n: int, tiles: int) -> None:
    """Fix the tiles per workgroup of the two-gate pass for (precision, n):
    1, 2, 4 or 8; 0 = tune again (qf_set_pass2_tiles)."""
    ctx = _ctx(device)
    nat.check(nat.load().qf_set_pass2_tiles(ctx, precision, n, tiles), ctx)


def set_batch_config(device, n_starts: int, slots: int, wg_per_cu: int = 1) -> None:
    """Fix the batched launch's shape for n_starts starts per block: slots
    (8 or 16) instantiations per workgroup, wg_per_cu workgroups per CU;
    slots = 0 = tune again (qf_set_batch_config)."""
    ctx = _ctx(device)
    nat.check(nat.load().qf_set_batch_config(ctx, n_starts, slots, wg_per_cu), ctx)


def _apply_kw(opt: nat.QfOptions, kw: dict):
    """Set option fields; gate_kinds (sequence of qf_gate_kind) becomes a
    ctypes array that the caller keeps alive for the call."""
    keep = None
    for k, v in kw.items():
        if k == "gate_kinds":
            if v is None:
                opt.gate_kinds = None
            else:
                a = np.ascontiguousarray(v, np.int32).reshape(-1)
                keep = (ctypes.c_int32 * max(1, a.size))(*a.tolist())
                opt.gate_kinds = ctypes.cast(keep, ctypes.POINTER(ctypes.c_int32))
        else:
            if not hasattr(opt, k):
                raise AttributeError(k)
            setattr(opt, k, v)
    return keep


def default_options(**kw) -> nat.QfOptions:
    o = nat.QfOptions()
    nat.load().qf_options_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def build(target: torch.Tensor, locs, gates: torch.Tensor, dtype=torch.complex128) -> torch.Tensor:
    """InitCircuitTensor: (S, N, N) builders G_p ... G_1 V^dagger."""
    N = target.shape[0]
    n = _n_of(N)
    locs = np.asarray(locs, np.int32).reshape(-1, 2)
    S, p = gates.shape[0], gates.shape[1]
    _c128(target, (N, N))
    _c128(gates, (S, p, 4, 4))
    X = torch.empty((S, N, N), dtype=dtype, device=target.device)
    ctx = _ctx(target.device)
    nat.check(nat.load().qf_build(ctx, n, _ptr(target), p, _loc(locs), _ptr(gates), S, _prec(X), _ptr(X)), ctx)
    return X


def apply_gate(builder: torch.Tensor, loc, gates: torch.Tensor, side: int, dagger: bool = False) -> torch.Tensor:
    """In place: X <- G X (side=QF_LEFT) or X G (QF_RIGHT), G^dagger if dagger."""
    S, n = _check_builder(builder)
    _c128(gates, (S, 4, 4))
    ctx = _ctx(builder.device)
    nat.check(nat.load().qf_apply_gate(ctx, n, S, _ptr(builder), _prec(builder), _loc(loc), _ptr(gates),
                                       int(side), int(bool(dagger))), ctx)
    return builder


def environment(builder: torch.Tensor, loc) -> torch.Tensor:
    """(S, 4, 4) complex128: partial trace of each builder over all qubits but loc."""
    S, n = _check_builder(builder)
    env = torch.empty((S, 4, 4), dtype=torch.complex128, device=builder.device)
    ctx = _ctx(builder.device)
    nat.check(nat.load().qf_environment(ctx, n, S, _ptr(builder), _prec(builder), _loc(loc), _ptr(env)), ctx)
    return env


def optimize_gate(env: torch.Tensor, u_old: torch.Tensor, beta: float = 0.0) -> torch.Tensor:
    count = env.shape[0]
    _c128(env, (count, 4, 4))
    _c128(u_old, (count, 4, 4))
    out = torch.empty_like(u_old)
    ctx = _ctx(env.device)
    nat.check(nat.load().qf_optimize_gate(ctx, count, _ptr(env), _ptr(u_old), float(beta), _ptr(out)), ctx)
    return out


def update_gate(builder: torch.Tensor, loc, half: int, gates: torch.Tensor, beta: float = 0.0,
                want_env: bool = False):
    """One TwoSidedSweep update in place; returns (gates, env or None)."""
    S, n = _check_builder(builder)
    _c128(gates, (S, 4, 4))
    env = torch.empty((S, 4, 4), dtype=torch.complex128, device=builder.device) if want_env else None
    ctx = _ctx(builder.device)
    nat.check(nat.load().qf_update_gate(ctx, n, S, _ptr(builder), _prec(builder), _loc(loc), int(half),
                                        float(beta), _ptr(gates), _ptr(env)), ctx)
    return gates, env


def cost(builder: torch.Tensor):
    """(costs (S,) float64, traces (S,) complex128) from the builders' traces."""
    S, n = _check_builder(builder)
    c = torch.empty((S,), dtype=torch.float64, device=builder.device)
    tr = torch.empty((S,), dtype=torch.complex128, device=builder.device)
    ctx = _ctx(builder.device)
    nat.check(nat.load().qf_cost(ctx, n, S, _ptr(builder), _prec(builder),
                                 ctypes.cast(ctypes.c_void_p(c.data_ptr()), ctypes.POINTER(ctypes.c_double)),
                                 _ptr(tr)), ctx)
    return c, tr


@dataclass
class Result:
    gates: torch.Tensor          # (p, 4, 4) best start
    all_gates: torch.Tensor      # (S, p, 4, 4)
    costs: np.ndarray            # (S,) FP64 costs of the returned gates
    best_start: int
    sweeps: int
    status: int
    n_resets: int
    n_rechecks: int
    mode_used: int
    elapsed_ms: float
    history: np.ndarray = field(default_factory=lambda: np.zeros((0, 0)))
    timing: dict = field(default_factory=dict)


def workspace_size(n: int, p: int, S: int, opt: nat.QfOptions) -> int:
    return int(nat.load().qf_workspace_size(n, p, S, ctypes.byref(opt)))


def instantiate(target: torch.Tensor, locs, init_gates: torch.Tensor, tol: float = 1e-10,
                options: nat.QfOptions | None = None, history_rows: int = 0,
                workspace: torch.Tensor | None = None, timing: bool = False, noalloc: bool = False,
                **kw) -> Result:
    """QFactor multistart instantiation (qf_instantiate); gate_kinds=[...]
    selects restricted gate kinds (QF_KIND_*).  noalloc=True calls
    qf_instantiate_noalloc instead (the library's fixed workspace; no
    `workspace` argument)."""
    opt = options if options is not None else default_options()
    _kinds_keep = _apply_kw(opt, kw)  # noqa: F841
    N = target.shape[0]
    n = _n_of(N)
    locs = np.asarray(locs, np.int32).reshape(-1, 2)
    S, p = init_gates.shape[0], init_gates.shape[1]
    _c128(target, (N, N))
    _c128(init_gates, (S, p, 4, 4))
    lib = nat.load()
    need = int(lib.qf_workspace_size(n, p, S, ctypes.byref(opt)))
    if need == 0:
        # invalid sizes or options: let the library reject them with its message
        need = 1
    if noalloc:
        workspace = None
    elif workspace is None or workspace.numel() < need:
        workspace = torch.empty((need,), dtype=torch.uint8, device=target.device)
    out = torch.empty((p, 4, 4), dtype=torch.complex128, device=target.device)
    out_all = torch.empty((S, p, 4, 4), dtype=torch.complex128, device=target.device)
    costs = (ctypes.c_double * S)()
    st = nat.QfStats()
    hist = None
    if history_rows > 0:
        hist = np.full((history_rows, S), np.nan, dtype=np.float64)
        st.cost_history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        st.cost_history_rows = history_rows
    st.timing = 1 if timing else 0
    ctx = _ctx(target.device)
    if noalloc:
        rc = lib.qf_instantiate_noalloc(ctx, n, _ptr(target), p, _loc(locs), _ptr(init_gates), S, float(tol),
                                        ctypes.byref(opt), _ptr(out), _ptr(out_all), costs, ctypes.byref(st))
    else:
        rc = lib.qf_instantiate(ctx, n, _ptr(target), p, _loc(locs), _ptr(init_gates), S, float(tol),
                                ctypes.byref(opt), _ptr(workspace), need, _ptr(out), _ptr(out_all), costs,
                                ctypes.byref(st))
    if rc not in (nat.QF_OK, nat.QF_ENUMERIC):
        nat.check(rc, ctx)
    h = hist[: min(history_rows, st.sweeps + 1)] if hist is not None else np.zeros((0, S))
    tm = dict(pass_ms=st.pass_ms, pass_launches=st.pass_launches, env_ms=st.env_ms,
              env_launches=st.env_launches, sweep_ms=st.sweep_ms, pass_tcols=st.pass_tcols,
              pass2_ms=st.pass2_ms, pass2_launches=st.pass2_launches) if timing \
        else dict(pass_tcols=st.pass_tcols)
    return Result(out, out_all, np.array(costs[:]), st.best_start, st.sweeps, st.status, st.n_resets,
                  st.n_rechecks, st.mode_used, st.elapsed_ms, h, tm)


def optimize_gate3(env: torch.Tensor, u_old: torch.Tensor, beta: float = 0.0) -> torch.Tensor:
    """The 8 x 8 gate update (qf_optimize_gate3) for (count, 8, 8) c128 environments."""
    count = env.shape[0]
    _c128(env, (count, 8, 8))
    _c128(u_old, (count, 8, 8))
    out = torch.empty_like(u_old)
    ctx = _ctx(env.device)
    nat.check(nat.load().qf_optimize_gate3(ctx, count, _ptr(env), _ptr(u_old), float(beta), _ptr(out)), ctx)
    return out


def instantiate3(target: torch.Tensor, locs, init_gates: torch.Tensor, tol: float = 1e-10,
                 options: nat.QfOptions | None = None, history_rows: int = 0, **kw) -> Result:
    """QFactor multistart instantiation of a circuit of three-qubit gates
    (qf_instantiate3): locs (p, 3), init_gates (S, p, 8, 8) c128."""
    opt = options if options is not None else default_options()
    _kinds_keep = _apply_kw(opt, kw)  # noqa: F841
    N = target.shape[0]
    n = _n_of(N)
    locs = np.asarray(locs, np.int32).reshape(-1, 3)
    S, p = init_gates.shape[0], init_gates.shape[1]
    _c128(target, (N, N))
    _c128(init_gates, (S, p, 8, 8))
    lib = nat.load()
    need = int(lib.qf_workspace_size3(n, p, S, ctypes.byref(opt)))
    if need == 0:
        need = 1  # invalid sizes or options: the library rejects them with its message
    workspace = torch.empty((need,), dtype=torch.uint8, device=target.device)
    out = torch.empty((p, 8, 8), dtype=torch.complex128, device=target.device)
    out_all = torch.empty((S, p, 8, 8), dtype=torch.complex128, device=target.device)
    costs = (ctypes.c_double * S)()
    st = nat.QfStats()
    hist = None
    if history_rows > 0:
        hist = np.full((history_rows, S), np.nan, dtype=np.float64)
        st.cost_history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        st.cost_history_rows = history_rows
    ctx = _ctx(target.device)
    rc = lib.qf_instantiate3(ctx, n, _ptr(target), p, _loc(locs), _ptr(init_gates), S, float(tol),
                             ctypes.byref(opt), _ptr(workspace), need, _ptr(out), _ptr(out_all), costs,
                             ctypes.byref(st))
    if rc not in (nat.QF_OK, nat.QF_ENUMERIC):
        nat.check(rc, ctx)
    h = hist[: min(history_rows, st.sweeps + 1)] if hist is not None else np.zeros((0, S))
    return Result(out, out_all, np.array(costs[:]), st.best_start, st.sweeps, st.status, st.n_resets,
                  st.n_rechecks, st.mode_used, st.elapsed_ms, h, dict(pass_tcols=st.pass_tcols))


@dataclass
class BatchResult:
    gates: torch.Tensor          # flat: per block, n_starts x p_b x 4 x 4 (every start's final gates)
    gate_offsets: np.ndarray     # (n_blocks + 1,)
    n_starts: int
    costs: np.ndarray            # (n_blocks, S) FP64 costs of the returned gates
    best: np.ndarray             # (n_blocks,)
    status: np.ndarray           # (n_blocks,)
    sweeps: np.ndarray           # (n_blocks,)
    elapsed_ms: float
    kernel_ms: float
    slots: int = 0                # instantiations per workgroup of the launch
    wg_per_cu: int = 0            # its workgroups per compute unit

    def block_gates(self, b: int) -> torch.Tensor:
        """(S, p_b, 4, 4) view of block b's gates."""
        g0, g1 = int(self.gate_offsets[b]), int(self.gate_offsets[b + 1])
        S = self.n_starts
        return self.gates[S * g0:S * g1].view(S, g1 - g0, 4, 4)


def pack_batch(targets, locs, init_gates):
    """Concatenate per-block targets (N_b x N_b), locations (p_b x 2) and
    initial gates (S x p_b x 4 x 4) into the flat layout of
    qf_instantiate_batch."""
    block_n = np.array([_n_of(t.shape[0]) for t in targets], np.int32)
    counts = [int(np.asarray(l).reshape(-1, 2).shape[0]) for l in locs]
    gate_offsets = np.zeros(len(counts) + 1, np.int32)
    gate_offsets[1:] = np.cumsum(counts)
    loc_flat = np.concatenate([np.asarray(l, np.int32).reshape(-1, 2) for l in locs])
    tflat = torch.cat([t.reshape(-1) for t in targets])
    gflat = torch.cat([g.reshape(-1, 4, 4) for g in init_gates])
    return block_n, gate_offsets, loc_flat, tflat, gflat


def batch_workspace_size(block_n, gate_offsets, S: int, opt: nat.QfOptions) -> int:
    bn = np.ascontiguousarray(block_n, np.int32)
    go = np.ascontiguousarray(gate_offsets, np.int32)
    return int(nat.load().qf_batch_workspace_size(len(bn), bn.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                                  go.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), S,
                                                  ctypes.byref(opt)))


def instantiate_batch(block_n, gate_offsets, locations, targets: torch.Tensor, init_gates: torch.Tensor,
                      n_starts: int, tol: float = 1e-10, options: nat.QfOptions | None = None,
                      workspace: torch.Tensor | None = None, out_gates: torch.Tensor | None = None,
                      timing: bool = False, **kw) -> BatchResult:
    """Batched QFactor over many small blocks (qf_instantiate_batch); the
    arguments are in the flat layout that pack_batch produces."""
    opt = options if options is not None else default_options()
    _kinds_keep = _apply_kw(opt, kw)  # noqa: F841
    bn = np.ascontiguousarray(block_n, np.int32)
    go = np.ascontiguousarray(gate_offsets, np.int32)
    lf = np.ascontiguousarray(locations, np.int32).reshape(-1)
    nb = len(bn)
    if targets.dtype != torch.complex128 or init_gates.dtype != torch.complex128:
        raise TypeError("targets and init_gates must be complex128")
    if not (targets.is_contiguous() and init_gates.is_contiguous()):
        raise ValueError("targets and init_gates must be contiguous")
    lib = nat.load()
    i32p = ctypes.POINTER(ctypes.c_int32)
    need = int(lib.qf_batch_workspace_size(nb, bn.ctypes.data_as(i32p), go.ctypes.data_as(i32p), n_starts,
                                           ctypes.byref(opt))) if nb > 0 else 0
    if need == 0:
        need = 1  # invalid sizes or options: the library rejects them with its message
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty((need,), dtype=torch.uint8, device=targets.device)
    if out_gates is None:
        out_gates = torch.empty_like(init_gates)
    costs = np.zeros((max(nb, 1), n_starts), np.float64)
    best = np.zeros(max(nb, 1), np.int32)
    status = np.zeros(max(nb, 1), np.int32)
    sweeps = np.zeros(max(nb, 1), np.int32)
    st = nat.QfStats()
    st.timing = 1 if timing else 0
    ctx = _ctx(targets.device)
    rc = lib.qf_instantiate_batch(ctx, nb, bn.ctypes.data_as(i32p), go.ctypes.data_as(i32p), lf.ctypes.data_as(i32p),
                                  _ptr(targets), _ptr(init_gates), n_starts, float(tol), ctypes.byref(opt),
                                  _ptr(workspace), need, _ptr(out_gates),
                                  costs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), best.ctypes.data_as(i32p),
                                  status.ctypes.data_as(i32p), sweeps.ctypes.data_as(i32p), ctypes.byref(st))
    nat.check(rc, ctx)
    return BatchResult(out_gates, go, n_starts, costs[:nb], best[:nb], status[:nb], sweeps[:nb], st.elapsed_ms,
                       st.sweep_ms, st.batch_slots, st.batch_wg_per_cu)


# ------------------------------------------------------------------ gradient

def _gates4(gates: torch.Tensor) -> tuple[torch.Tensor, bool]:
    if gates.dim() == 3:
        return gates.unsqueeze(0), True
    return gates, False


def gradient(target: torch.Tensor, locs, gates: torch.Tensor, precision: int = nat.QF_C128,
             workspace: torch.Tensor | None = None):
    """Cost and gate gradient (qf_gradient): gates (S, p, 4, 4) or (p, 4, 4)
    complex128; returns cost (S,) float64 and grad (same shape as gates),
    grad = dDelta/dRe u + i dDelta/dIm u."""
    g4, squeeze = _gates4(gates)
    N = target.shape[0]
    n = _n_of(N)
    locs = np.asarray(locs, np.int32).reshape(-1, 2)
    S, p = g4.shape[0], g4.shape[1]
    _c128(target, (N, N))
    _c128(g4, (S, p, 4, 4))
    lib = nat.load()
    need = int(lib.qf_gradient_workspace_size(n, p, S, precision)) or 1
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty((need,), dtype=torch.uint8, device=target.device)
    cost_t = torch.empty((S,), dtype=torch.float64, device=target.device)
    grad = torch.empty_like(g4)
    ctx = _ctx(target.device)
    nat.check(lib.qf_gradient(ctx, n, _ptr(target), p, _loc(locs), _ptr(g4), S, precision, _ptr(workspace), need,
                              _ptr(cost_t), _ptr(grad)), ctx)
    if squeeze:
        return cost_t[0], grad[0]
    return cost_t, grad


def cost_of_gates(target: torch.Tensor, locs, gates: torch.Tensor, precision: int = nat.QF_C128) -> torch.Tensor:
    """Cost of gate sets without a gradient: builders from qf_build, costs
    from qf_cost.  gates (S, p, 4, 4) -> (S,) float64, or (p, 4, 4) -> scalar."""
    g4, squeeze = _gates4(gates)
    X = build(target, locs, g4.contiguous(), torch.complex64 if precision == nat.QF_C64 else torch.complex128)
    c, _ = cost(X)
    return c[0] if squeeze else c


class _CostFn(torch.autograd.Function):
    """Delta(gates) with the backward from qf_gradient (forward and gradient
    are taken together when the gates need a gradient, and the gradient is
    kept for the backward; otherwise only the cost is computed)."""

    @staticmethod
    def forward(ctx, gates, target, locs, precision):
        if not ctx.needs_input_grad[0]:
            return cost_of_gates(target, locs, gates.detach(), precision)
        c, G = gradient(target, locs, gates.detach(), precision)
        ctx.save_for_backward(G)
        return c

    @staticmethod
    def backward(ctx, gout):
        (G,) = ctx.saved_tensors
        shape = (-1,) + (1,) * (G.dim() - 1) if G.dim() == 4 else ()
        return gout.reshape(shape).to(G.dtype) * G, None, None, None


def cost_fn(gates: torch.Tensor, target: torch.Tensor, locs, precision: int = nat.QF_C128) -> torch.Tensor:
    """Differentiable cost: gates (S, p, 4, 4) -> (S,) (or (p, 4, 4) -> scalar)."""
    return _CostFn.apply(gates, target, np.asarray(locs, np.int32).reshape(-1, 2), precision)


def su4_gates(theta: torch.Tensor) -> torch.Tensor:
    """exp(i H(theta)) for theta (..., 15) float64 on the GPU (qf_su4_gates)."""
    th = theta.contiguous()
    if th.dtype != torch.float64:
        raise TypeError("theta must be float64")
    count = th.numel() // 15
    out = torch.empty(th.shape[:-1] + (4, 4), dtype=torch.complex128, device=th.device)
    ctx = _ctx(th.device)
    nat.check(nat.load().qf_su4_gates(ctx, count, _ptr(th), _ptr(out)), ctx)
    return out


def su4_vjp(theta: torch.Tensor, grad_gates: torch.Tensor) -> torch.Tensor:
    """dtheta_k = Re Tr(grad^dagger dU/dtheta_k) (qf_su4_vjp)."""
    th = theta.contiguous()
    gg = grad_gates.contiguous().to(torch.complex128)
    count = th.numel() // 15
    out = torch.empty_like(th)
    ctx = _ctx(th.device)
    nat.check(nat.load().qf_su4_vjp(ctx, count, _ptr(th), _ptr(gg), _ptr(out)), ctx)
    return out


class _SU4Fn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta):
        ctx.save_for_backward(theta)
        return su4_gates(theta.detach())

    @staticmethod
    def backward(ctx, gout):
        (theta,) = ctx.saved_tensors
        return su4_vjp(theta.detach(), gout)


def su4(theta: torch.Tensor) -> torch.Tensor:
    """Differentiable theta -> exp(i H(theta))."""
    return _SU4Fn.apply(theta)


def lbfgs_options(**kw) -> nat.QfLbfgsOptions:
    o = nat.QfLbfgsOptions()
    nat.load().qf_lbfgs_options_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


@dataclass
class LbfgsResult:
    theta: torch.Tensor      # (S, p, 15)
    costs: np.ndarray        # (S,)
    best_start: int
    iterations: int
    status: int
    evaluations: int
    elapsed_ms: float
    history: np.ndarray = field(default_factory=lambda: np.zeros((0, 0)))


def lbfgs(target: torch.Tensor, locs, theta0: torch.Tensor, tol: float = 1e-10, history_rows: int = 0,
          options: nat.QfLbfgsOptions | None = None, **kw) -> LbfgsResult:
    """L-BFGS over parameterised SU(4) gates (qf_lbfgs); theta0 (S, p, 15)."""
    opt = options if options is not None else lbfgs_options()
    for k, v in kw.items():
        setattr(opt, k, v)
    th = theta0.contiguous()
    if th.dim() == 2:
        th = th.unsqueeze(0)
    if th.dtype != torch.float64:
        raise TypeError("theta0 must be float64")
    N = target.shape[0]
    n = _n_of(N)
    locs = np.asarray(locs, np.int32).reshape(-1, 2)
    S, p = th.shape[0], th.shape[1]
    _c128(target, (N, N))
    lib = nat.load()
    need = int(lib.qf_lbfgs_workspace_size(n, p, S, ctypes.byref(opt))) or 1
    workspace = torch.empty((need,), dtype=torch.uint8, device=target.device)
    out = torch.empty_like(th)
    costs = (ctypes.c_double * S)()
    st = nat.QfLbfgsResult()
    hist = None
    if history_rows > 0:
        hist = np.full((history_rows, S), np.nan, dtype=np.float64)
        st.cost_history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        st.cost_history_rows = history_rows
    ctx = _ctx(target.device)
    nat.check(lib.qf_lbfgs(ctx, n, _ptr(target), p, _loc(locs), _ptr(th), S, float(tol), ctypes.byref(opt),
                           _ptr(workspace), need, _ptr(out), costs, ctypes.byref(st)), ctx)
    h = hist[: min(history_rows, st.iterations + 1)] if hist is not None else np.zeros((0, S))
    return LbfgsResult(out, np.array(costs[:]), st.best_start, st.iterations, st.status, st.evaluations,
                       st.elapsed_ms, h)


@dataclass
class DeletionResult:
    keep: np.ndarray         # (p,) 1 kept, 0 deleted
    gates: torch.Tensor      # (kept, 4, 4) the final circuit's gates in order
    locs: np.ndarray         # (kept, 2)
    cost: float              # FP64 cost of the final circuit
    attempts: int
    deleted: int
    sweeps: int
    elapsed_ms: float


def delete_gates(target: torch.Tensor, locs, gates: torch.Tensor, pool: torch.Tensor, tol: float = 1e-10,
                 options: nat.QfOptions | None = None, **kw) -> DeletionResult:
    """Uni-directional gate-deletion sweep (qf_delete_gates): gates (p, 4, 4)
    realise target on `locs`; pool (S, p, 4, 4) seeds starts 1..S-1."""
    opt = options if options is not None else default_options()
    _kinds_keep = _apply_kw(opt, kw)  # noqa: F841
    N = target.shape[0]
    n = _n_of(N)
    locs = np.asarray(locs, np.int32).reshape(-1, 2)
    p = locs.shape[0]
    S = pool.shape[0]
    _c128(target, (N, N))
    _c128(gates, (p, 4, 4))
    _c128(pool, (S, p, 4, 4))
    lib = nat.load()
    need = int(lib.qf_delete_gates_workspace_size(n, p, S, ctypes.byref(opt))) or 1
    workspace = torch.empty((need,), dtype=torch.uint8, device=target.device)
    out = torch.empty((p, 4, 4), dtype=torch.complex128, device=target.device)
    keep = (ctypes.c_int32 * p)()
    cost_out = ctypes.c_double()
    st = nat.QfDeleteResult()
    ctx = _ctx(target.device)
    nat.check(lib.qf_delete_gates(ctx, n, _ptr(target), p, _loc(locs), _ptr(gates), _ptr(pool), S, float(tol),
                                  ctypes.byref(opt), _ptr(workspace), need, keep, _ptr(out),
                                  ctypes.byref(cost_out), ctypes.byref(st)), ctx)
    km = np.array(keep[:], np.int32)
    kcount = int(km.sum())
    return DeletionResult(km, out[:kcount].clone(), locs[km == 1], float(cost_out.value), st.attempts,
                          st.deleted, st.sweeps, st.elapsed_ms)
