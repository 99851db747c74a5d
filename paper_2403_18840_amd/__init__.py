"""Python binding of the dmc C ABI (include/dmc.h): argument marshalling only.

Every step of the hot path runs in the library's HIP kernels; torch is used for device memory
and streams.  Importing this module does not need a GPU; calls that launch kernels do, and they
fail loudly if the library is not built.
"""
from __future__ import annotations

import ctypes
from typing import NamedTuple
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdmc.so")

DMC_OK = 0
STATUS = {0: "DMC_OK", -1: "DMC_E_INVALID", -2: "DMC_E_NOMEM", -3: "DMC_E_DEVICE", -4: "DMC_E_COMPILE",
          -5: "DMC_E_STATE", -6: "DMC_E_NUMERIC"}
D_MU, D_LAMBDA, D_K = 1, 2, 4
SAMPLER_UNIFORM, SAMPLER_VEGAS = 0, 1
ROUTING_PATH, ROUTING_BLOCKS = 0, 1
GENERATE_ENUMERATE, GENERATE_CONSTRUCT = 0, 1

# every symbol include/dmc.h declares
ABI_SYMBOLS = [
    "dmc_last_error", "dmc_version", "dmc_compile_graph", "dmc_graph_query", "dmc_graph_set_importance",
    "dmc_graph_export_diagrams",
    "dmc_graph_source", "dmc_graph_root_orders", "dmc_graph_destroy", "dmc_accum_create", "dmc_accum_reset", "dmc_accum_destroy",
    "dmc_sampler_create", "dmc_sample", "dmc_sampler_get_grid", "dmc_sampler_set_grid", "dmc_sampler_refine",
    "dmc_vegas_refine",
    "dmc_sampler_read_histogram", "dmc_sampler_destroy", "dmc_eval_batch", "dmc_eval_accumulate_noalloc",
    "dmc_accumulate", "dmc_estimate",
    "dmc_accum_read", "dmc_flow_create", "dmc_flow_create_spline", "dmc_flow_param_count", "dmc_flow_set_params", "dmc_flow_get_params",
    "dmc_flow_sample", "dmc_flow_log_density", "dmc_flow_walk", "dmc_flow_train_step", "dmc_flow_destroy",
    "dmc_chains_create", "dmc_chains_step", "dmc_chains_step_walk", "dmc_chains_read", "dmc_chains_reset",
    "dmc_chains_destroy",
    "dmc_chains_training_data",
    "dmc_effective_mass", "dmc_probe", "dmc_combine_iterations", "dmc_chains_ratio", "dmc_mass_table",
    "dmc_checkpoint_save", "dmc_checkpoint_load", "dmc_proposal_select", "dmc_chains_run",
]


class DmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class GraphSpec(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("deriv_mask", ctypes.c_uint32), ("diagram_index", ctypes.c_int32),
                ("part_size", ctypes.c_int32), ("taylor_order", ctypes.c_int32), ("deriv_k", ctypes.c_int32),
                ("routing", ctypes.c_int32), ("spin_deg", ctypes.c_int32), ("generation", ctypes.c_int32)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("dim", ctypes.c_int32), ("n_diagrams", ctypes.c_int32),
                ("n_root_classes", ctypes.c_int32), ("n_momenta", ctypes.c_int32), ("n_g_leaves", ctypes.c_int32),
                ("n_v_leaves", ctypes.c_int32), ("n_groups", ctypes.c_int32), ("n_parts", ctypes.c_int32),
                ("part_size", ctypes.c_int32), ("ops_sample", ctypes.c_int64 * 4),
                ("ops_k", ctypes.c_int64 * 4), ("ops_naive", ctypes.c_int64 * 4),
                ("ops_sample_exec", ctypes.c_int64 * 4), ("ops_k_exec", ctypes.c_int64 * 4),
                ("n_roots", ctypes.c_int32), ("taylor_order", ctypes.c_int32),
                ("ops_k_deriv", ctypes.c_int64 * 4), ("ops_k_deriv_exec", ctypes.c_int64 * 4),
                ("deriv_k", ctypes.c_int32), ("routing", ctypes.c_int32), ("spin_deg", ctypes.c_int32),
                ("generation", ctypes.c_int32)]


class Instance(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("mu", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("gamma", ctypes.c_double)]


_lib = None

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
U64 = ctypes.c_uint64
F64 = ctypes.c_double


def lib():
    """Load libdmc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch ships its own HIP runtime with the same soname; load it first so that the library
    # binds to that one runtime instead of bringing a second one into the process
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "dmc_last_error": (ctypes.c_char_p, []),
        "dmc_version": (ctypes.c_char_p, []),
        "dmc_compile_graph": (I32, [ctypes.POINTER(GraphSpec), ctypes.POINTER(P)]),
        "dmc_graph_query": (I32, [P, ctypes.POINTER(GraphInfo)]),
        "dmc_graph_set_importance": (I32, [P, I32]),
        "dmc_graph_export_diagrams": (I32, [P, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
        "dmc_graph_source": (I32, [P, I32, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
        "dmc_graph_destroy": (None, [P]),
        "dmc_graph_root_orders": (I32, [P, P, I32]),
        "dmc_accum_create": (I32, [I32, I32, I32, ctypes.POINTER(P)]),
        "dmc_accum_reset": (I32, [P, P]),
        "dmc_accum_destroy": (None, [P]),
        "dmc_sampler_create": (I32, [I32, I32, I32, F64, F64, ctypes.POINTER(P)]),
        "dmc_sample": (I32, [P, U64, U64, I64, P, I64, P, P]),
        "dmc_sampler_get_grid": (I32, [P, P]),
        "dmc_sampler_set_grid": (I32, [P, P, P]),
        "dmc_sampler_refine": (I32, [P, F64, P]),
        "dmc_sampler_read_histogram": (I32, [P, P, P]),
        "dmc_sampler_destroy": (None, [P]),
        "dmc_eval_batch": (I32, [P, P, I32, P, I32, P, I64, P, I64, P, P, P, P]),
        "dmc_eval_accumulate_noalloc": (I32, [P, P, I32, P, I32, P, I64, P, I64, P, P, P, P]),
        "dmc_combine_iterations": (I32, [I32, I32, P, P, P, P, P]),
        "dmc_proposal_select": (I32, [I32, P, P, F64, F64, I64, F64, ctypes.POINTER(I32), ctypes.POINTER(F64)]),
        "dmc_chains_ratio": (I32, [I32, I32, I32, I32, P, I32, P, I32, P, P]),
        "dmc_mass_table": (I32, [I32, P, I32, P, F64, P, P, P, P, P]),
        "dmc_checkpoint_save": (I32, [P, P, P, U64, U64, P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t), P]),
        "dmc_checkpoint_load": (I32, [P, P, P, ctypes.POINTER(U64), ctypes.POINTER(U64), P, ctypes.c_size_t, P]),
        "dmc_accumulate": (I32, [P, P, P, P]),
        "dmc_estimate": (I32, [P, P, P, ctypes.POINTER(I64), ctypes.POINTER(I64), P]),
        "dmc_accum_read": (I32, [P, P, ctypes.POINTER(I64), P]),
        "dmc_flow_create": (I32, [I32, I32, P, ctypes.POINTER(P)]),
        "dmc_flow_create_spline": (I32, [I32, I32, P, ctypes.POINTER(P)]),
        "dmc_flow_param_count": (I32, [P, ctypes.POINTER(I64)]),
        "dmc_flow_set_params": (I32, [P, P, P]),
        "dmc_flow_get_params": (I32, [P, P, P]),
        "dmc_flow_sample": (I32, [P, P, U64, U64, I64, P, I64, P, P, P, F64, F64, P]),
        "dmc_flow_log_density": (I32, [P, P, I64, I64, P, P]),
        "dmc_flow_train_step": (I32, [P, P, I64, U64, U64, I64, P, F64, P, ctypes.POINTER(F64), P]),
        "dmc_flow_destroy": (None, [P]),
        "dmc_chains_create": (I32, [I64, I32, I32, I32, I32, I32, ctypes.POINTER(P)]),
        "dmc_chains_step": (I32, [P, P, I64, P, P, I64, I64, F64, U64, I32, P]),
        "dmc_chains_step_walk": (I32, [P, P, I64, P, P, P, P, I64, F64, U64, I32, P]),
        "dmc_flow_walk": (I32, [P, P, P, I64, I64, F64, U64, U64, P, I64, P, P, P, P, F64, F64, P]),
        "dmc_probe": (I32, [I32, I64, ctypes.POINTER(F64), ctypes.POINTER(F64), P]),
        "dmc_vegas_refine": (I32, [I32, I32, P, P, F64, P]),
        "dmc_chains_training_data": (I32, [P, P, I64, P, P]),
        "dmc_chains_read": (I32, [P, P, ctypes.POINTER(I64), ctypes.POINTER(I64), P]),
        "dmc_chains_run": (I32, [P, P, P, I32, P, I32, P, P, F64, F64, U64, U64, I64, I64, F64, U64, U64, P, I64, P, P,
                                 P, P, P]),
        "dmc_chains_reset": (I32, [P, P]),
        "dmc_chains_destroy": (None, [P]),
        "dmc_effective_mass": (I32, [I32, F64, I32, P, P, P, P, P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(st, allow=()):
    if st != DMC_OK and st not in allow:
        raise DmcError(st, lib().dmc_last_error().decode())
    return st


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t, dtype_name, what):
    """Device pointer of a contiguous CUDA tensor of the given dtype (or None)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a device tensor")
    if str(t.dtype) != "torch." + dtype_name:
        raise TypeError(f"{what} must be {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def dim(order: int) -> int:
    return 4 * order - 1


def coupling(rs: float) -> float:
    """gamma = alpha r_s, alpha = (4 / (9 pi))^(1/3): the Yukawa strength 8 pi gamma / (q^2 + lambda) in units
    k_F = E_F = 1 (e^2 = 2 Ry a_0, k_F = 1 / (alpha r_s a_0))."""
    return (4.0 / (9.0 * math.pi)) ** (1.0 / 3.0) * rs


class Graph:
    """A compiled diagram graph (dmc_compile_graph)."""

    def __init__(self, order: int, deriv_mask: int = 0, diagram_index: int = -1, part_size: int = 0,
                 taylor_order: int = 0, deriv_k: int = 0, routing: int = 0, spin_deg: int = 2, generation: int = 0):
        self.h = P()
        spec = GraphSpec(order, deriv_mask, diagram_index, part_size, taylor_order, deriv_k, routing, spin_deg,
                         generation)
        _check(lib().dmc_compile_graph(ctypes.byref(spec), ctypes.byref(self.h)))
        self.order = order
        self.deriv_mask = deriv_mask
        self.taylor_order = taylor_order
        self.routing = routing
        self.n_roots = self.info().n_roots
        self.importance_roots = 1

    def root_orders(self):
        """[(m, l, e)] per root: d^m/dmu^m d^l/dlambda^l (d/dk)^e of the self-energy."""
        buf = (I32 * (3 * self.n_roots))()
        _check(lib().dmc_graph_root_orders(self.h, buf, 3 * self.n_roots))
        return [tuple(buf[3 * r: 3 * r + 3]) for r in range(self.n_roots)]

    def set_importance(self, n_roots: int):
        """dmc_graph_set_importance: the leading roots whose |w| eval_batch sums into imp_out (1: the value)."""
        _check(lib().dmc_graph_set_importance(self.h, int(n_roots)))
        self.importance_roots = int(n_roots)

    def info(self) -> GraphInfo:
        gi = GraphInfo()
        _check(lib().dmc_graph_query(self.h, ctypes.byref(gi)))
        return gi

    def _text(self, fn, *pre):
        n = ctypes.c_size_t()
        _check(fn(self.h, *pre, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value + 1)
        _check(fn(self.h, *pre, buf, n.value + 1, ctypes.byref(n)))
        return buf.value.decode()

    def export(self) -> str:
        return self._text(lib().dmc_graph_export_diagrams)

    def source(self, n_groups: int = 1) -> str:
        return self._text(lib().dmc_graph_source, I32(n_groups))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.dmc_graph_destroy(self.h)
            self.h = None


class Accumulator:
    """FP64 running sums (dmc_accum_*)."""

    def __init__(self, n_groups: int, n_k: int, n_roots: int = 1):
        self.h = P()
        _check(lib().dmc_accum_create(n_groups, n_k, n_roots, ctypes.byref(self.h)))
        self.n_groups, self.n_k, self.n_roots = n_groups, n_k, n_roots

    def reset(self, stream=None):
        _check(lib().dmc_accum_reset(self.h, _stream(stream)))

    def read(self, stream=None):
        import numpy as np
        out = np.zeros((self.n_groups, self.n_roots, self.n_k, 2, 2), dtype=np.float64)
        n = I64()
        _check(lib().dmc_accum_read(self.h, out.ctypes.data_as(P), ctypes.byref(n), _stream(stream)))
        return out, n.value

    def estimate(self, n_inst: int, stream=None):
        """(mean, stderr) as complex arrays [n_inst][n_roots][n_k], plus (n_samples, n_nonfinite)."""
        import numpy as np
        m = np.zeros((n_inst, self.n_roots, self.n_k, 2))
        e = np.zeros_like(m)
        ns, nf = I64(), I64()
        _check(lib().dmc_estimate(self.h, m.ctypes.data_as(P), e.ctypes.data_as(P), ctypes.byref(ns),
                                  ctypes.byref(nf), _stream(stream)), allow=(-6,))
        return m[..., 0] + 1j * m[..., 1], e[..., 0] + 1j * e[..., 1], ns.value, nf.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.dmc_accum_destroy(self.h)
            self.h = None


class Sampler:
    """Philox4x32-10 sampler through a VEGAS grid (or uniform) and the physical map."""

    def __init__(self, kind: int, order: int, n_bins: int = 50, beta: float = 25.0, qmax: float = 6.0):
        self.h = P()
        _check(lib().dmc_sampler_create(kind, order, n_bins, beta, qmax, ctypes.byref(self.h)))
        self.kind, self.order, self.dim = kind, order, dim(order)
        self.n_bins = n_bins if kind == SAMPLER_VEGAS else 1
        self.beta, self.qmax = beta, qmax

    def sample(self, seed: int, first: int, x, jac, stream=None):
        n = jac.numel()
        ld = x.shape[1]
        if x.dim() != 2 or x.shape[0] != self.dim:
            raise ValueError(f"x must be [{self.dim}, ld]")
        _check(lib().dmc_sample(self.h, seed, first, n, _dptr(x, "float32", "x"), ld, _dptr(jac, "float32", "jac"),
                                _stream(stream)))

    def grid(self):
        import numpy as np
        e = np.zeros((self.dim, self.n_bins + 1))
        _check(lib().dmc_sampler_get_grid(self.h, e.ctypes.data_as(P)))
        return e

    def set_grid(self, edges, stream=None):
        import numpy as np
        e = np.ascontiguousarray(edges, dtype=np.float64)
        _check(lib().dmc_sampler_set_grid(self.h, e.ctypes.data_as(P), _stream(stream)))

    def refine(self, alpha: float = 0.5, stream=None):
        _check(lib().dmc_sampler_refine(self.h, alpha, _stream(stream)))

    def histogram(self, stream=None):
        import numpy as np
        h = np.zeros((self.dim, self.n_bins))
        _check(lib().dmc_sampler_read_histogram(self.h, h.ctypes.data_as(P), _stream(stream)))
        return h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.dmc_sampler_destroy(self.h)
            self.h = None


def instances(params):
    """params: iterable of (beta, mu, lambda, gamma) -> ctypes array of dmc_instance."""
    params = list(params)
    arr = (Instance * len(params))(*[Instance(*p) for p in params])
    return arr


def eval_batch(graph: Graph, inst, k_ext, x, jac, acc: Accumulator, f_out=None, imp_out=None, stream=None):
    """dmc_eval_batch: inst is a list of (beta, mu, lambda, gamma); k_ext host floats."""
    import numpy as np
    arr = instances(inst)
    k = np.ascontiguousarray(k_ext, dtype=np.float32)
    n = jac.numel()
    if x.dim() != 2:
        raise ValueError("x must be [D, ld]")
    _check(lib().dmc_eval_batch(graph.h, arr, len(arr), k.ctypes.data_as(P), len(k), _dptr(x, "float32", "x"),
                                x.shape[1], _dptr(jac, "float32", "jac"), n, acc.h,
                                _dptr(f_out, "float32", "f_out"), _dptr(imp_out, "float32", "imp_out"),
                                _stream(stream)))


def eval_accumulate_noalloc(graph: Graph, inst, k_ext, x, jac, acc: Accumulator, f_out=None, imp_out=None,
                            stream=None):
    """dmc_eval_accumulate_noalloc: eval_batch + accumulate with the library's static device scratch (the
    graph's kernel must have been loaded by an eval_batch call)."""
    import numpy as np
    arr = instances(inst)
    k = np.ascontiguousarray(k_ext, dtype=np.float32)
    if x.dim() != 2:
        raise ValueError("x must be [D, ld]")
    _check(lib().dmc_eval_accumulate_noalloc(graph.h, arr, len(arr), k.ctypes.data_as(P), len(k),
                                             _dptr(x, "float32", "x"), x.shape[1], _dptr(jac, "float32", "jac"),
                                             jac.numel(), acc.h, _dptr(f_out, "float32", "f_out"),
                                             _dptr(imp_out, "float32", "imp_out"), _stream(stream)))


def accumulate(acc: Accumulator, sampler: Sampler | None = None, imp=None, stream=None):
    _check(lib().dmc_accumulate(acc.h, sampler.h if sampler is not None else None,
                                _dptr(imp, "float32", "imp"), _stream(stream)))


def sigma_function():
    """torch.autograd.Function around eval_batch with derivative roots.

    apply(mu, lam, k, graph, x, jac, beta, gamma) -> Sigma estimate [K, 2] (Re, Im) in float64,
    where mu, lam are 0-dim float64 tensors and k a 1-D float64 tensor (host).  The graph must be
    compiled with deriv_mask = D_MU | D_LAMBDA | D_K.  One device pass produces the value and the
    three derivative estimates (the samples do not depend on the parameters); backward contracts
    the saved derivatives with the incoming gradient."""
    import torch

    class SigmaFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, mu, lam, k, graph, x, jac, beta, gamma):
            if graph.deriv_mask != (D_MU | D_LAMBDA | D_K):
                raise ValueError("graph must carry all three derivative roots")
            ks = k.detach().cpu().numpy().astype("float32")
            acc = Accumulator(1, len(ks), 4)
            eval_batch(graph, [(float(beta), float(mu), float(lam), float(gamma))], ks, x, jac, acc)
            accumulate(acc)
            m, e, ns, nf = acc.estimate(1)
            import numpy as np
            ri = torch.from_numpy(np.stack([m[0].real, m[0].imag], axis=-1))  # [4, K, 2]
            ctx.save_for_backward(ri[1], ri[2], ri[3])
            return ri[0].clone()

        @staticmethod
        def backward(ctx, g):
            dmu, dlam, dk = ctx.saved_tensors
            return (g * dmu).sum(), (g * dlam).sum(), (g * dk).sum(-1), None, None, None, None, None

    return SigmaFn


def _n_groups(inst):
    lams = []
    for p in inst:
        if p[2] not in lams:
            lams.append(p[2])
    return len(lams)


def adapt_grid(graph: Graph, inst, k_ext, sampler: Sampler, n_samples: int, iters: int, seed: int = 1,
               first: int = 0, alpha: float = 0.5):
    """`iters` VEGAS refinements of the sampler's grid on batches of `n_samples` points (the samples
    are discarded).  Returns the next unused sample index."""
    import numpy as np
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    D = dim(graph.order)
    acc = Accumulator(_n_groups(inst), len(k_ext), graph.n_roots)
    X = torch.empty((D, n_samples), dtype=torch.float32, device=dev)
    J = torch.empty(n_samples, dtype=torch.float32, device=dev)
    imp = torch.empty(n_samples, dtype=torch.float32, device=dev)
    ks = np.asarray(k_ext, dtype=np.float32)
    for _ in range(iters):
        acc.reset()
        sampler.sample(seed, first, X, J)
        eval_batch(graph, inst, ks, X, J, acc, imp_out=imp)
        accumulate(acc, sampler, imp)
        sampler.refine(alpha)
        first += n_samples
    return first


def train_flow(graph: Graph, inst, k_ext, sampler: Sampler, flow: "Flow", epochs: int = 8, steps: int = 16,
               minibatch: int = 1 << 17, lr: float = 1e-3, alpha: float = 0.85, uniform: float = 0.05, seed: int = 3,
               anneal=None):
    """Fit `flow` (on the VEGAS coordinates of `sampler`, whose grid stays frozen) to the absolute
    integrand by the weighted forward KL of Appendix A, with Adam on the device.

    Every step draws `minibatch` new points, evaluates the graph on them (the training weight of a
    point is its importance value, sum |f| J over the graph's importance roots (the value alone unless
    Graph.set_importance adds derivative roots) over the proposal density) and takes one step.  The
    first epoch draws from the grid alone; later epochs from the mixture alpha q_flow + uniform
    q_uniform + (rest) q_grid of the current flow, so the training points follow the flow as it
    sharpens.  k_ext selects the external momenta whose |Sigma| integrand the flow learns (the figure
    of merit's).  anneal: a list of one beta per epoch (Appendix A's annealing in temperature: start hot,
    where the integrand is smoother, and cool to the target); every epoch then trains on the integrand at
    its beta through a sampler of that beta with the same grid (the flow lives on the grid coordinates,
    where tau = beta u, so what it learns carries over).  Returns the loss of the last step of every epoch."""
    import numpy as np
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    D = dim(graph.order)
    if flow.dim != D:
        raise ValueError("flow dimension does not match the graph's order")
    ks = np.asarray(k_ext, dtype=np.float32)
    acc = Accumulator(_n_groups(inst), len(ks), graph.n_roots)
    X = torch.empty((D, minibatch), dtype=torch.float32, device=dev)
    J = torch.empty(minibatch, dtype=torch.float32, device=dev)
    U = torch.empty((D, minibatch), dtype=torch.float32, device=dev)
    imp = torch.empty(minibatch, dtype=torch.float32, device=dev)
    if anneal is not None and len(anneal) != epochs:
        raise ValueError("anneal needs one beta per epoch")
    losses = []
    step = 0
    for ep in range(epochs):
        loss = None
        s_ep, inst_ep = sampler, inst
        if anneal is not None:
            b_ep = float(anneal[ep])
            s_ep = Sampler(SAMPLER_VEGAS, graph.order, n_bins=sampler.n_bins, beta=b_ep, qmax=sampler.qmax)
            s_ep.set_grid(sampler.grid())
            inst_ep = [(b_ep,) + tuple(p[1:]) for p in inst]
        for b in range(steps):
            first = step * minibatch
            last = b == steps - 1
            if ep == 0:
                s_ep.sample(seed, first, X, J)
                eval_batch(graph, inst_ep, ks, X, J, acc, imp_out=imp)
                loss = flow.train_step(imp, seed=seed, first=first, lr=lr, want_loss=last)
            else:
                flow.sample(s_ep, seed, first, X, J, u_out=U, alpha=alpha, uniform=uniform)
                eval_batch(graph, inst_ep, ks, X, J, acc, imp_out=imp)
                loss = flow.train_step(imp, u=U, lr=lr, want_loss=last)
            acc.reset()
            step += 1
        losses.append(loss)
    return losses


def integrate(graph: Graph, inst, k_ext, n_samples: int, iters: int, adapt: int = 5, seed: int = 1,
              kind: int = SAMPLER_VEGAS, n_bins: int = 50, beta: float = 25.0, qmax: float = 6.0, alpha: float = 0.5,
              flow: "Flow | None" = None, flow_alpha: float = 0.85, flow_uniform: float = 0.05,
              train: dict | None = None, train_k=None, fallback: float | None = 1.0, report: dict | None = None):
    """Importance-sampling estimate of Sigma (and derivative roots) with the library's sampler.

    `adapt` iterations refine the VEGAS grid (their samples are discarded).  With a `flow`, it is
    then trained on the frozen grid (`train`: keyword arguments of train_flow, on the external
    momenta train_k, default all; None skips training) and the estimate draws from the mixture
    flow_alpha q_flow + flow_uniform q_uniform + (rest) q_grid.  The next `iters`
    iterations accumulate into one FP64 accumulator, whose mean over all estimation samples is the
    estimate.  Returns (mean, stderr) complex [n_inst][n_roots][K].

    Fallback to VEGAS (with a flow and `fallback` not None): one probe iteration of each proposal, on points
    of their own that are discarded like the adaptation's, decides through dmc_proposal_select whether the
    flow beats the grid by the factor `fallback` in variance times time; if not, or if its probe dropped a
    non-finite weight, the estimate draws from the grid.  A flow iteration that drops a non-finite weight
    switches the remaining iterations to the grid (the switch depends on earlier iterations only, so each
    iteration's estimate stays unbiased).  `report`, a dict, receives "proposal" ("flow" or "vegas"),
    "gain" and "switched_at" (the iteration of a switch, or None)."""
    import numpy as np
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    ks = np.asarray(k_ext, dtype=np.float32)
    D = dim(graph.order)
    s = Sampler(kind, graph.order, n_bins, beta, qmax)
    first = 0
    if kind == SAMPLER_VEGAS:
        first = adapt_grid(graph, inst, ks, s, n_samples, adapt, seed=seed, alpha=alpha)
    if flow is not None:
        if kind != SAMPLER_VEGAS:
            raise ValueError("the flow maps onto a VEGAS grid")
        if train is not None:
            kt = ks if train_k is None else np.asarray(train_k, dtype=np.float32)
            opts = dict({"seed": seed + 1, "alpha": flow_alpha, "uniform": flow_uniform}, **train)
            train_flow(graph, inst, kt, s, flow, **opts)
    acc = Accumulator(_n_groups(inst), len(ks), graph.n_roots)
    X = torch.empty((D, n_samples), dtype=torch.float32, device=dev)
    J = torch.empty(n_samples, dtype=torch.float32, device=dev)
    use_flow, gain, switched = flow is not None, None, None
    if use_flow and fallback is not None:
        errs, times, nfs = [], [], []
        for which in ("flow", "grid"):
            pacc = Accumulator(_n_groups(inst), len(ks), graph.n_roots)
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record()
            if which == "flow":
                flow.sample(s, seed + 4, 0, X, J, alpha=flow_alpha, uniform=flow_uniform)
            else:
                s.sample(seed + 5, 0, X, J)
            eval_batch(graph, inst, ks, X, J, pacc)
            accumulate(pacc)
            t1.record()
            t1.synchronize()
            _, e, _, nf = pacc.estimate(len(inst))
            errs.append(np.stack([e[:, 0].real, e[:, 0].imag]))
            times.append(t0.elapsed_time(t1))
            nfs.append(nf)
        use_flow, gain = proposal_select(errs[0], errs[1], times[0], times[1], nfs[0], fallback)
    est_seed = seed + 2 if use_flow else seed
    for it in range(iters):
        if use_flow:
            flow.sample(s, est_seed, first, X, J, alpha=flow_alpha, uniform=flow_uniform)
        else:
            s.sample(seed, first, X, J)
        eval_batch(graph, inst, ks, X, J, acc)
        accumulate(acc)
        first += n_samples
        if use_flow and fallback is not None and it + 1 < iters and acc.estimate(len(inst))[3] > 0:
            use_flow, switched = False, it + 1
    m, e, ns, nf = acc.estimate(len(inst))
    if report is not None:
        report.update(proposal="flow" if use_flow else "vegas", gain=gain, switched_at=switched)
    return m, e


class Flow:
    """Coupling flow on the VEGAS coordinates (dmc_flow_*): kind "affine" (dmc_flow_create: affine couplings,
    BF16 matrix cores) or "spline" (dmc_flow_create_spline: the paper's rational-quadratic spline couplings,
    uniform base)."""

    def __init__(self, dim_: int, masks, kind: str = "affine"):
        import numpy as np
        m = np.ascontiguousarray(masks, dtype=np.int8)
        self.h = P()
        if kind not in ("affine", "spline"):
            raise ValueError("kind must be 'affine' or 'spline'")
        create = lib().dmc_flow_create if kind == "affine" else lib().dmc_flow_create_spline
        _check(create(dim_, m.shape[0], m.ctypes.data_as(P), ctypes.byref(self.h)))
        self.dim, self.n_layers, self.masks, self.kind = dim_, m.shape[0], m, kind
        n = I64()
        _check(lib().dmc_flow_param_count(self.h, ctypes.byref(n)))
        self.n_params = n.value

    def set_params(self, theta, stream=None):
        import numpy as np
        t = np.ascontiguousarray(theta, dtype=np.float32)
        if t.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        _check(lib().dmc_flow_set_params(self.h, t.ctypes.data_as(P), _stream(stream)))

    def params(self, stream=None):
        import numpy as np
        t = np.empty(self.n_params, dtype=np.float32)
        _check(lib().dmc_flow_get_params(self.h, t.ctypes.data_as(P), _stream(stream)))
        return t

    def sample(self, sampler: Sampler, seed: int, first: int, x, jac, u_out=None, lq_out=None, alpha: float = 1.0,
               uniform: float = 0.0, stream=None):
        """Mixture alpha q_flow + (1 - alpha - uniform) q_grid + uniform q_uniform (dmc_flow_sample)."""
        n = jac.numel()
        _check(lib().dmc_flow_sample(self.h, sampler.h, seed, first, n, _dptr(x, "float32", "x"), x.shape[1],
                                     _dptr(jac, "float32", "jac"), _dptr(u_out, "float32", "u_out"),
                                     _dptr(lq_out, "float32", "lq_out"), alpha, uniform, _stream(stream)))

    def walk(self, sampler: Sampler, u_state, sigma: float, seed: int, first: int, x, jac, jac_flow, u_out,
             jac_flow_state, alpha: float = 1.0, uniform: float = 0.0, stream=None):
        """Base-space random-walk proposals from the states u_state [D][>= n] (dmc_flow_walk, spline flows):
        x, jac (1/q of the mixture alpha, uniform), jac_flow (1/q_T), u_out [D][>= n] at the proposals, and
        jac_flow_state (1/q_T at the states)."""
        n = jac.numel()
        _check(lib().dmc_flow_walk(self.h, sampler.h, _dptr(u_state, "float32", "u_state"), u_state.shape[1], n,
                                   sigma, seed, first, _dptr(x, "float32", "x"), x.shape[1],
                                   _dptr(jac, "float32", "jac"), _dptr(jac_flow, "float32", "jac_flow"),
                                   _dptr(u_out, "float32", "u_out"), _dptr(jac_flow_state, "float32", "jac_flow_state"),
                                   alpha, uniform, _stream(stream)))

    def log_density(self, u, lq, stream=None):
        _check(lib().dmc_flow_log_density(self.h, _dptr(u, "float32", "u"), u.shape[1], lq.numel(),
                                          _dptr(lq, "float32", "lq"), _stream(stream)))

    def train_step(self, w, u=None, seed: int = 0, first: int = 0, lr: float = 0.0, grad_out=None,
                   want_loss: bool = True, stream=None):
        n = w.numel()
        loss = F64()
        _check(lib().dmc_flow_train_step(self.h, _dptr(u, "float32", "u"), u.shape[1] if u is not None else n,
                                         seed, first, n, _dptr(w, "float32", "w"), lr,
                                         _dptr(grad_out, "float32", "grad_out"),
                                         ctypes.byref(loss) if want_loss else None, _stream(stream)))
        return loss.value if want_loss else None

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.dmc_flow_destroy(self.h)
            self.h = None


class Chains:
    """Independent-proposal Markov chains, one per sample lane (dmc_chains_*), their sums kept per chain
    batch (batch b: chains [b n // n_batches, (b + 1) n // n_batches))."""

    def __init__(self, n: int, n_groups: int, n_k: int, n_roots: int = 1, n_batches: int = 1, dim_u: int = 0):
        self.h = P()
        _check(lib().dmc_chains_create(n, n_batches, n_groups, n_k, n_roots, dim_u, ctypes.byref(self.h)))
        self.n, self.n_groups, self.n_k, self.n_roots, self.n_batches = n, n_groups, n_k, n_roots, n_batches
        self.dim_u = dim_u
        self.S = n_groups * n_roots * n_k * 2

    def step(self, f_prop, jac_prop, alpha: float, seed: int, offset: int = 0, measure: bool = True, u_prop=None,
             stream=None):
        """f_prop: the f_out capture of eval_batch at the proposals (flat [G][R][K][2][ld]); jac_prop: 1/q;
        u_prop: [dim_u][ld_u] coordinates (chains that keep them); chain c takes proposal (c + offset) mod n."""
        if self.dim_u and (u_prop is None or u_prop.dim() != 2 or u_prop.shape[0] != self.dim_u
                           or u_prop.shape[1] < self.n):
            raise ValueError(f"u_prop must be [{self.dim_u}][>= {self.n}]")
        ld = f_prop.numel() // self.S
        if f_prop.numel() != ld * self.S or ld < self.n:
            raise ValueError(f"f_prop must hold [{self.S}][ld >= {self.n}] values, got {f_prop.numel()}")
        if jac_prop.numel() < self.n:
            raise ValueError(f"jac_prop must hold at least {self.n} values")
        _check(lib().dmc_chains_step(self.h, _dptr(f_prop, "float32", "f_prop"), ld,
                                     _dptr(jac_prop, "float32", "jac_prop"), _dptr(u_prop, "float32", "u_prop"),
                                     u_prop.shape[1] if u_prop is not None else 0, offset, alpha, seed,
                                     1 if measure else 0, _stream(stream)))

    def step_walk(self, f_prop, jac_prop, jac_flow_prop, jac_flow_state, u_prop, alpha: float, seed: int,
                  measure: bool = True, stream=None):
        """A base-space random-walk step (dmc_chains_step_walk): chain c's proposal is column c of the
        output of Flow.walk, evaluated by eval_batch into f_prop."""
        ld = f_prop.numel() // self.S
        if f_prop.numel() != ld * self.S or ld < self.n:
            raise ValueError(f"f_prop must hold [{self.S}][ld >= {self.n}] values, got {f_prop.numel()}")
        if min(jac_prop.numel(), jac_flow_prop.numel(), jac_flow_state.numel()) < self.n:
            raise ValueError(f"the weights must hold at least {self.n} values")
        if u_prop.dim() != 2 or u_prop.shape[0] != self.dim_u or u_prop.shape[1] < self.n:
            raise ValueError(f"u_prop must be [{self.dim_u}][>= {self.n}]")
        _check(lib().dmc_chains_step_walk(self.h, _dptr(f_prop, "float32", "f_prop"), ld,
                                          _dptr(jac_prop, "float32", "jac_prop"),
                                          _dptr(jac_flow_prop, "float32", "jac_flow_prop"),
                                          _dptr(jac_flow_state, "float32", "jac_flow_state"),
                                          _dptr(u_prop, "float32", "u_prop"), u_prop.shape[1], alpha, seed,
                                          1 if measure else 0, _stream(stream)))

    def training_data(self, u_out, w_out, stream=None):
        """States as forward-KL training data: u_out [dim_u][>= n] coordinates, w_out [n] = p / pi."""
        if w_out.numel() < self.n or (self.dim_u and (u_out.dim() != 2 or u_out.shape[0] != self.dim_u
                                                      or u_out.shape[1] < self.n)):
            raise ValueError("u_out must be [dim_u][>= n] and w_out hold n values")
        _check(lib().dmc_chains_training_data(self.h, _dptr(u_out, "float32", "u_out"),
                                              u_out.shape[1] if u_out is not None else 0,
                                              _dptr(w_out, "float32", "w_out"), _stream(stream)))

    def read(self, stream=None):
        """(sums [n_batches][S + 1][2] float64, states measured, proposals accepted)."""
        import numpy as np
        sums = np.zeros((self.n_batches, self.S + 1, 2), dtype=np.float64)
        nm, na = I64(), I64()
        _check(lib().dmc_chains_read(self.h, sums.ctypes.data_as(P), ctypes.byref(nm), ctypes.byref(na),
                                     _stream(stream)))
        return sums, nm.value, na.value

    def reset(self, stream=None):
        _check(lib().dmc_chains_reset(self.h, _stream(stream)))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.dmc_chains_destroy(self.h)
            self.h = None


class McmcResult(NamedTuple):
    """mean, err: complex [n_inst][n_roots][K] (ratio estimate over all measured steps and chains; error
    from the scatter of the independent chain batches).  acceptance: over the measured steps.
    is_mean, is_err: plain importance sampling over every proposal (thermalisation included).
    halves: ((mean, err) of the first half of the measured steps, the same of the second half, z of
    their difference per entry): chains still relaxing from the proposal density show as a trend
    between the halves, which the batch error does not see."""
    mean: object
    err: object
    acceptance: float
    is_mean: object
    is_err: object
    halves: tuple


def mcmc_integrate(graph: Graph, inst, k_ext, sampler: Sampler, n_chains: int, steps: int, thermal: int = 200,
                   alpha: float = 0.5, seed: int = 1, n_batches: int = 32, flow: "Flow | None" = None,
                   flow_alpha: float = 0.85, flow_uniform: float = 0.05, walk_every: int = 0,
                   walk_sigma: float = 0.05) -> McmcResult:
    """Markov-chain estimate (eq. nf_mcmc_estimator_qft_final_revised) with independent proposals from
    `sampler` (its grid frozen) or, with `flow`, from the flow's mixture.  Every step draws n_chains
    proposals and hands chain c proposal (c + r) mod n_chains with r uniform and fresh (the
    mixture orders its draws by component).  The first `thermal` steps are discarded: chains start
    from the proposal density, and an independence sampler whose proposal is far from |f| needs many
    steps to reach the target.  Every later step is measured.  With a spline `flow` and walk_every = m > 0,
    every m-th step after the first is instead a random-walk move in the flow's base space (Flow.walk,
    step size walk_sigma); its proposals stay out of the importance-sampling estimate."""
    import numpy as np
    import torch
    if steps < 2:
        raise ValueError("steps must be at least 2")
    if n_batches < 2:
        raise ValueError("n_batches must be at least 2 for an error estimate")
    dev = torch.device("cuda", torch.cuda.current_device())
    ks = np.asarray(k_ext, dtype=np.float32)
    K = len(ks)
    G = _n_groups(inst)
    R = graph.n_roots
    D = dim(graph.order)
    walk = walk_every > 0
    if walk and (flow is None or flow.kind != "spline"):
        raise ValueError("the base-space walk needs a spline flow")
    ch = Chains(n_chains, G, K, R, n_batches, dim_u=D if walk else 0)
    acc = Accumulator(G, K, R)
    X = torch.empty((D, n_chains), dtype=torch.float32, device=dev)
    J = torch.empty(n_chains, dtype=torch.float32, device=dev)
    F = torch.empty(G * R * K * 2 * n_chains, dtype=torch.float32, device=dev)
    if walk:
        U = torch.empty((D, n_chains), dtype=torch.float32, device=dev)
        US = torch.empty((D, n_chains), dtype=torch.float32, device=dev)
        JF = torch.empty(n_chains, dtype=torch.float32, device=dev)
        JFS = torch.empty(n_chains, dtype=torch.float32, device=dev)
        WS = torch.empty(n_chains, dtype=torch.float32, device=dev)
        acc_walk = Accumulator(G, K, R)  # walk proposals are no draws from q: kept out of the IS estimate
    if not walk:
        # the whole loop in the library (dmc_chains_run), in two halves for the trend check
        arr = instances(inst)
        kk = np.ascontiguousarray(ks, dtype=np.float32)
        h1 = steps // 2

        def run(first, n_thermal, n_steps, key):
            _check(lib().dmc_chains_run(ch.h, graph.h, arr, len(arr), kk.ctypes.data_as(P), len(kk), sampler.h,
                                        flow.h if flow is not None else None, flow_alpha, flow_uniform, seed, first,
                                        n_thermal, n_steps, alpha, seed + 0x5EED, key, _dptr(X, "float32", "x"),
                                        X.shape[1], _dptr(J, "float32", "jac"), _dptr(F, "float32", "f"), None,
                                        acc.h, _stream(None)))
        run(0, thermal, h1, seed ^ 0x0FF5E7)
        half = ch.read()[0]
        run((thermal + h1) * n_chains, 0, steps - h1, (seed ^ 0x0FF5E7) + 0x100000000)
        offsets = ()
    else:
        offsets = np.random.default_rng([seed, 0x0FF5E7]).integers(0, n_chains, size=thermal + steps)
        half = None
    for t in range(len(offsets)):
        if walk and t > 0 and t % walk_every == walk_every - 1:
            ch.training_data(US, WS)
            flow.walk(sampler, US, walk_sigma, seed + 0x3A1C, t * n_chains, X, J, JF, U, JFS, alpha=flow_alpha,
                      uniform=flow_uniform)
            eval_batch(graph, inst, ks, X, J, acc_walk, f_out=F)
            accumulate(acc_walk)
            ch.step_walk(F, J, JF, JFS, U, alpha, seed + 0x5EED, measure=t >= thermal)
        else:
            if flow is not None:
                flow.sample(sampler, seed, t * n_chains, X, J, u_out=U if walk else None, alpha=flow_alpha,
                            uniform=flow_uniform)
            else:
                sampler.sample(seed, t * n_chains, X, J)
            eval_batch(graph, inst, ks, X, J, acc, f_out=F)
            accumulate(acc)
            ch.step(F, J, alpha, seed + 0x5EED, offset=int(offsets[t]), measure=t >= thermal,
                    u_prop=U if walk else None)
        if t + 1 == thermal:
            ch.reset()  # the acceptance rate counts the measured steps only
        if t + 1 == thermal + steps // 2:
            half = ch.read()[0]
    sums, _, accepted = ch.read()
    S = G * R * K * 2
    lam_of = []
    for p in inst:
        if p[2] not in lam_of:
            lam_of.append(p[2])

    def ratio(sm):
        # the ratio estimator with its batch errors and the r_s rescaling, in the library (dmc_chains_ratio)
        return chains_ratio(sm, G, R, K, graph.order, inst)

    m, e = ratio(sums)
    m1, e1 = ratio(half)
    m2, e2 = ratio(sums - half)
    z = np.empty_like(m)
    with np.errstate(invalid="ignore", divide="ignore"):
        z.real = (m1.real - m2.real) / np.hypot(e1.real, e2.real)
        z.imag = (m1.imag - m2.imag) / np.hypot(e1.imag, e2.imag)
    mi, ei, _, _ = acc.estimate(len(inst))
    return McmcResult(m, e, accepted / (n_chains * steps), mi, ei, ((m1, e1), (m2, e2), z))



def chains_ratio(sums, n_groups: int, n_roots: int, n_k: int, order: int, inst):
    """dmc_chains_ratio: (mean, err) complex [n_inst][n_roots][n_k] of the Markov-chain ratio estimator from batch
    sums [n_batches][S + 1][2] (dmc_chains_read), with each instance's (gamma / gamma_group)^order."""
    import numpy as np
    sm = np.ascontiguousarray(sums, dtype=np.float64)
    arr = instances(inst)
    m = np.zeros((len(inst), n_roots, n_k, 2))
    e = np.zeros_like(m)
    _check(lib().dmc_chains_ratio(sm.shape[0], n_groups, n_roots, n_k, sm.ctypes.data_as(P), order, arr, len(arr),
                                  m.ctypes.data_as(P), e.ctypes.data_as(P)))
    return m[..., 0] + 1j * m[..., 1], e[..., 0] + 1j * e[..., 1]


def combine_iterations(means, errs):
    """dmc_combine_iterations: equal-weight combination of iteration estimates [n_iter][...] (real arrays): returns
    (mean, err, chi2_dof) of the trailing shape."""
    import numpy as np
    mm = np.ascontiguousarray(means, dtype=np.float64)
    ee = np.ascontiguousarray(errs, dtype=np.float64)
    if mm.shape != ee.shape or mm.ndim < 1:
        raise ValueError("means and errs must have one shape [n_iter, ...]")
    nv = int(np.prod(mm.shape[1:])) if mm.ndim > 1 else 1
    out = [np.empty(nv) for _ in range(3)]
    _check(lib().dmc_combine_iterations(mm.shape[0], nv, mm.ctypes.data_as(P), ee.ctypes.data_as(P),
                                        *[o.ctypes.data_as(P) for o in out]))
    return tuple(o.reshape(mm.shape[1:]) for o in out)


def proposal_select(err_flow, err_grid, t_flow: float, t_grid: float, nonfinite_flow: int, min_gain: float = 1.0):
    """dmc_proposal_select: (use_flow, gain) from the standard errors (real arrays of one shape) and times of one
    probe iteration of the flow mixture and of the VEGAS grid."""
    import numpy as np
    ef = np.ascontiguousarray(err_flow, dtype=np.float64).reshape(-1)
    eg = np.ascontiguousarray(err_grid, dtype=np.float64).reshape(-1)
    if ef.shape != eg.shape:
        raise ValueError("err_flow and err_grid must have one shape")
    use, gain = I32(), F64()
    _check(lib().dmc_proposal_select(ef.size, ef.ctypes.data_as(P), eg.ctypes.data_as(P), t_flow, t_grid,
                                     nonfinite_flow, min_gain, ctypes.byref(use), ctypes.byref(gain)))
    return bool(use.value), gain.value


def mass_table(order: int, root_orders, est, beta: float):
    """dmc_mass_table: {(n, m, l): value} tables (sigma, a, b) of one order from its roots' estimates at k_F
    (complex [n_roots])."""
    import numpy as np
    ro = np.ascontiguousarray(np.asarray(root_orders, dtype=np.int32).reshape(-1))
    R = ro.size // 3
    ev = np.ascontiguousarray(np.stack([np.real(est), np.imag(est)], axis=-1), dtype=np.float64)
    nml = np.zeros(3 * R, dtype=np.int32)
    sg, aa, bb = np.zeros(R), np.zeros(R), np.zeros(R)
    n_out = I32()
    _check(lib().dmc_mass_table(order, ro.ctypes.data_as(P), R, ev.ctypes.data_as(P), beta, nml.ctypes.data_as(P),
                                sg.ctypes.data_as(P), aa.ctypes.data_as(P), bb.ctypes.data_as(P), ctypes.byref(n_out)))
    keys = [tuple(int(v) for v in nml[3 * i: 3 * i + 3]) for i in range(n_out.value)]
    return ({k: float(sg[i]) for i, k in enumerate(keys)}, {k: float(aa[i]) for i, k in enumerate(keys)},
            {k: float(bb[i]) for i, k in enumerate(keys)})


def checkpoint_save(sampler=None, flow=None, acc=None, seed: int = 0, next_index: int = 0, stream=None) -> bytes:
    """dmc_checkpoint_save: the integration state (any of sampler, flow, accumulator, plus the Philox position) as
    bytes."""
    n = ctypes.c_size_t()
    hs = [h.h if h is not None else None for h in (sampler, flow, acc)]
    st = _stream(stream) if any(hs) else None   # the position alone touches no device
    _check(lib().dmc_checkpoint_save(*hs, seed, next_index, None, 0, ctypes.byref(n), st))
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().dmc_checkpoint_save(*hs, seed, next_index, buf, n.value, ctypes.byref(n), st))
    return buf.raw[: n.value]


def checkpoint_load(data: bytes, sampler=None, flow=None, acc=None, stream=None):
    """dmc_checkpoint_load into the given handles; returns (seed, next_index)."""
    sd, nx = U64(), U64()
    hs = [h.h if h is not None else None for h in (sampler, flow, acc)]
    st = _stream(stream) if any(hs) else None
    _check(lib().dmc_checkpoint_load(*hs, ctypes.byref(sd), ctypes.byref(nx), data, len(data), st))
    return sd.value, nx.value


def vegas_refine(edges, hist, alpha: float = 0.5):
    """dmc_vegas_refine: the VEGAS refinement of grid edges [D][B + 1] by a histogram [D][B], on the host."""
    import numpy as np
    e = np.ascontiguousarray(edges, dtype=np.float64)
    h = np.ascontiguousarray(hist, dtype=np.float64)
    if e.ndim != 2 or h.shape != (e.shape[0], e.shape[1] - 1):
        raise ValueError("edges must be [D][B + 1] and hist [D][B]")
    out = np.empty_like(e)
    _check(lib().dmc_vegas_refine(e.shape[0], h.shape[1], e.ctypes.data_as(P), h.ctypes.data_as(P), alpha,
                                  out.ctypes.data_as(P)))
    return out


def probe(kind: int, work: int, stream=None):
    """dmc_probe: (milliseconds of one launch, operations or bytes moved) of a throughput probe: kind 0
    FP32 FMA, 1 hardware 2^x, 2 hardware reciprocal (work = iterations), 3 device copy (work = bytes)."""
    ms, ops = F64(), F64()
    _check(lib().dmc_probe(kind, work, ctypes.byref(ms), ctypes.byref(ops), _stream(stream)))
    return ms.value, ops.value


def effective_mass(N: int, lambda_R: float, sigma_fs: dict, a: dict, b: dict):
    """dmc_effective_mass: tables {(n, m, l): value} of Re Sigma^(n,m,l)(k_F, i w_0), a^(n,m,l) and b^(n,m,l)
    (missing entries are zero).  Returns dict of float64 arrays [N + 1]: delta_mu, a_xi, b_xi, mass,
    mass_partial (m*/m through each order at xi = 1)."""
    import numpy as np
    keys = sorted(set(sigma_fs) | set(a) | set(b))
    nml = np.array(keys, dtype=np.int32).reshape(-1, 3)
    cols = [np.array([t.get(k, 0.0) for k in keys], dtype=np.float64) for t in (sigma_fs, a, b)]
    outs = {name: np.zeros(N + 1) for name in ("delta_mu", "a_xi", "b_xi", "mass", "mass_partial")}
    ptr = lambda arr: arr.ctypes.data_as(P)
    _check(lib().dmc_effective_mass(N, lambda_R, len(keys), ptr(nml), ptr(cols[0]), ptr(cols[1]), ptr(cols[2]),
                                    *(ptr(outs[k]) for k in ("delta_mu", "a_xi", "b_xi", "mass", "mass_partial"))))
    return outs


def mass_coefficients(N: int, rs: float, lambda_R: float, beta: float = 25.0, mu: float = 1.0, n_samples: int = 1 << 22,
                      batches: int = 16, adapt: int = 6, seed: int = 0x5E1F, qmax: float = 6.0, n_bins: int = 50):
    """Fermi-surface Taylor coefficients for the renormalised series to total order N (n + m + l <= N):
    per order n a graph with every d^m/dmu^m d^l/dlambda^l, m + l <= N - n, and their k derivatives
    (Sec. VI.A, eq. sigma_xi_dmu_dlambda and eq. deltam_partitions), integrated at k = k_F with a VEGAS
    grid adapted to that order.  Returns a list over `batches` independent batches of n_samples points
    of (sigma_fs, a, b) tables as dmc_effective_mass takes them."""
    import numpy as np
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    inst = [(beta, mu, lambda_R, coupling(rs))]
    ks = np.array([1.0], dtype=np.float32)
    tables = [({}, {}, {}) for _ in range(batches)]
    for n in range(1, N + 1):
        T = N - n
        g = Graph(n, D_MU | D_LAMBDA | D_K, taylor_order=T) if T > 0 else Graph(n, D_K)
        orders = g.root_orders()
        s = Sampler(SAMPLER_VEGAS, n, n_bins=n_bins, beta=beta, qmax=qmax)
        first = adapt_grid(g, inst, ks, s, n_samples, adapt, seed=seed + n)
        X = torch.empty((dim(n), n_samples), dtype=torch.float32, device=dev)
        J = torch.empty(n_samples, dtype=torch.float32, device=dev)
        acc = Accumulator(1, 1, g.n_roots)
        for bi in range(batches):
            acc.reset()
            s.sample(seed + n, first + bi * n_samples, X, J)
            eval_batch(g, inst, ks, X, J, acc)
            accumulate(acc)
            m_, _, _, _ = acc.estimate(1)
            ts, ta, tb = mass_table(n, orders, m_[0, :, 0], beta)
            for t, part in zip(tables[bi], (ts, ta, tb)):
                t.update(part)
    return tables


def effective_mass_estimate(N: int, rs: float, lambda_R: float, **kw):
    """m*/m of the renormalised series (Sec. VI.A) through orders 1..N with jackknife errors over the
    independent batches of mass_coefficients (the ratio is a nonlinear function of the coefficients).
    Returns (mass_partial [N + 1], its errors, delta_mu [N + 1], its errors)."""
    import numpy as np
    tables = mass_coefficients(N, rs, lambda_R, **kw)
    B = len(tables)

    def mean(sub):
        out = []
        for t in range(3):
            keys = set().union(*(tb[t].keys() for tb in sub))
            out.append({k: float(np.mean([tb[t].get(k, 0.0) for tb in sub])) for k in keys})
        return out

    full = effective_mass(N, lambda_R, *mean(tables))
    jk = [effective_mass(N, lambda_R, *mean(tables[:i] + tables[i + 1:])) for i in range(B)]
    err = {}
    for name in ("mass_partial", "delta_mu"):
        v = np.array([j[name] for j in jk])
        err[name] = np.sqrt((B - 1) / B * np.sum((v - v.mean(axis=0)) ** 2, axis=0))
    return full["mass_partial"], err["mass_partial"], full["delta_mu"], err["delta_mu"]



def train_flow_mcmc(graph: Graph, inst, k_ext, sampler: Sampler, flow: "Flow", rounds: int = 4,
                    n_chains: int = 1 << 17, thermal: int = 200, collect: int = 8, stride: int = 10,
                    steps: int = 64, lr: float = 1e-3, alpha: float = 0.0, flow_alpha: float = 0.85,
                    flow_uniform: float = 0.05, seed: int = 11):
    """Fit `flow` to |f| on samples generated by Markov chains (Appendix A's MCMC training data).

    Every round starts fresh chains whose independent proposals come from the current flow's mixture
    (the flow changes between rounds, so old states would carry a stale proposal density), targets
    pi = alpha q + (1 - alpha)|f|, discards `thermal` steps, then collects the states `collect` times
    every `stride` steps as points u' with weights p / pi (1 at alpha = 0).  `steps` Adam steps of the
    weighted forward KL follow, cycling through the collected sets.  Returns the mean loss of each round."""
    import numpy as np
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    D = dim(graph.order)
    if flow.dim != D:
        raise ValueError("flow dimension does not match the graph's order")
    ks = np.asarray(k_ext, dtype=np.float32)
    G, K, R = _n_groups(inst), len(ks), graph.n_roots
    acc = Accumulator(G, K, R)
    X = torch.empty((D, n_chains), dtype=torch.float32, device=dev)
    J = torch.empty(n_chains, dtype=torch.float32, device=dev)
    U = torch.empty((D, n_chains), dtype=torch.float32, device=dev)
    F = torch.empty(G * R * K * 2 * n_chains, dtype=torch.float32, device=dev)
    rng = np.random.default_rng([seed, 0x7A1])
    losses = []
    first = 0
    for r in range(rounds):
        ch = Chains(n_chains, G, K, R, 1, D)
        sets = []
        for t in range(thermal + collect * stride):
            flow.sample(sampler, seed, first, X, J, u_out=U, alpha=flow_alpha, uniform=flow_uniform)
            first += n_chains
            eval_batch(graph, inst, ks, X, J, acc, f_out=F)
            acc.reset()
            ch.step(F, J, alpha, seed + 0x5EED + r, offset=int(rng.integers(n_chains)), measure=False, u_prop=U)
            if t >= thermal and (t - thermal) % stride == stride - 1:
                Uc = torch.empty((D, n_chains), dtype=torch.float32, device=dev)
                Wc = torch.empty(n_chains, dtype=torch.float32, device=dev)
                ch.training_data(Uc, Wc)
                sets.append((Uc, Wc))
        ls = []
        for s_ in range(steps):
            Uc, Wc = sets[s_ % len(sets)]
            ls.append(flow.train_step(Wc, u=Uc, lr=lr, want_loss=(s_ % len(sets) == len(sets) - 1)))
        losses.append(float(np.mean([v for v in ls if v is not None])))
    return losses
