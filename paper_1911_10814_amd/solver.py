"""Python binding of the nested block solver: device memory and streams from
PyTorch, every computation in the HIP library (``libns_hip.so``).

``NsContext``       one mesh: symbolic set-up, workspace, assembly, solves.
``SolveOptions``    mirror of ``ns_solve_opts`` (paper defaults, Sec. 3.1).
``NestedSolveFn``   torch.autograd.Function R -> x(R) whose backward runs the
                    transposed nested solve (adjoint) on the device.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np
import torch

from . import _lib
from ._lib import NsError


@dataclasses.dataclass
class SolveOptions:
    rtol: float = 1e-8
    atol: float = 1e-50
    rtol_A: float = 1e-3
    rtol_S: float = 1e-3
    rtol_I: float = 1e-3
    m: int = 200
    nmax: int = 200
    m_A: int = 200
    nmax_A: int = 200
    m_S: int = 200
    nmax_S: int = 200
    pc_A: str = "amg"            # "amg" | "jacobi"
    pc_I: str | None = None      # P of the inner A-solves (Algorithm 2); None: as pc_A
    precision: str = "fp64"      # "fp64" | "fp32_inner"
    cheb_degree: int = 2
    cheb_degree_S: int = 0       # degree on the S_hat hierarchy (0: cheb_degree)
    cheb_ratio: float = 10.0     # smoother interval [lambda/cheb_ratio, lambda]
    cc_scale_A: float = 1.0      # AMG coarse-grid correction scaling, A hierarchy
    cc_scale_S: float = 1.0      # and S_hat hierarchy
    cycles_S: int = 1            # V-cycle iterations per application of P_S
    cycle_index_A: int = 1       # AMG cycle index below the finest level (1: V, 2: W), A hierarchy
    cycle_index_S: int = 1       # and S_hat hierarchy
    pc: str = "scr"              # outer preconditioner: "scr" (Algorithm 3) | "simple" (Sec. 3.2)
    schedule: list | None = None  # fixed iteration counts per Krylov call (replay)
    record: bool = True           # record the iteration count of every Krylov call

    def to_c(self):
        o = _lib.NsSolveOpts()
        for f in ("rtol", "atol", "rtol_A", "rtol_S", "rtol_I", "m", "nmax", "m_A", "nmax_A", "m_S", "nmax_S",
                  "cheb_degree", "cheb_degree_S", "cheb_ratio", "cycles_S", "cc_scale_A", "cc_scale_S",
                  "cycle_index_A", "cycle_index_S"):
            setattr(o, f, getattr(self, f))
        o.pc_A = {"amg": 0, "jacobi": 1}[self.pc_A]
        o.pc_I = {None: 0, "amg": 1, "jacobi": 2}[self.pc_I]
        o.precision = {"fp64": 0, "fp32_inner": 1}[self.precision]
        o.pc = {"scr": 0, "simple": 1}[self.pc]
        keep = []
        if self.schedule is not None:
            arr = np.ascontiguousarray(self.schedule, dtype=np.int32)
            keep.append(arr)
            o.h_sched = arr.ctypes.data_as(_lib.PI)
            o.sched_len = len(arr)
        out = None
        if self.record:
            out = np.zeros(1 << 16, dtype=np.int32)
            keep.append(out)
            o.h_sched_out = out.ctypes.data_as(_lib.PI)
            o.sched_cap = len(out)
        return o, keep, out


def _stream_handle(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


class NsContext:
    """A mesh bound to one GPU.

    ``case`` is any object with the fields of ``ns_inputs.Case`` (xyz, tets,
    mask, outlet_ptr, faces; n_nodes, n_elems, n_outlets)."""

    def __init__(self, case, *, max_m=200, max_m_A=200, max_m_S=200, coarse_nodes=128, max_levels=16,
                 coarse_matchings=3, device="cuda:0"):
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.N = int(case.n_nodes)
        self.n_out = int(case.n_outlets)
        self._xyz = np.ascontiguousarray(case.xyz, dtype=np.float64)
        self._tets = np.ascontiguousarray(case.tets, dtype=np.int32)
        self._optr = np.ascontiguousarray(case.outlet_ptr, dtype=np.int32)
        self._faces = np.ascontiguousarray(case.faces, dtype=np.int32).reshape(-1, 3)
        self._mask = np.ascontiguousarray(case.mask, dtype=np.uint8)
        mesh = _lib.NsMesh(self.N, int(case.n_elems), self.n_out, self._xyz.ctypes.data_as(_lib.PD),
                           self._tets.ctypes.data_as(_lib.PI), self._optr.ctypes.data_as(_lib.PI),
                           self._faces.ctypes.data_as(_lib.PI),
                           self._mask.ctypes.data_as(C.POINTER(C.c_uint8)))
        opts = _lib.NsCtxOpts(max_m, max_m_A, max_m_S, coarse_nodes, max_levels, coarse_matchings)
        handle = C.c_void_p()
        nbytes = C.c_size_t()
        st = self.lib.ns_ctx_create(C.byref(mesh), C.byref(opts), C.byref(handle), C.byref(nbytes))
        if st != 0:
            raise NsError(st, self.lib.ns_last_error(None).decode())
        self.h = handle
        self.workspace_bytes = int(nbytes.value)
        self.ws = None
        self.sizes = self.query()
        self.nnzb = self.sizes[1]

    # ------------------------------------------------------------------ basics
    def _check(self, st):
        if st < 0:
            raise NsError(st, self.lib.ns_last_error(self.h).decode())
        return st

    def query(self):
        out = (C.c_int64 * 6)()
        self._check(self.lib.ns_query(self.h, out))
        return list(out)

    def layout(self):
        """Finest-level layout: dict with the fixed-width row width the FP32 planes may take
        (0: none), whether 16-bit column offsets are available, and what the bound context uses."""
        out = (C.c_int32 * 4)()
        self._check(self.lib.ns_query_layout(self.h, out))
        return {"ell": out[0], "col16_available": bool(out[1]), "ell_bound": bool(out[2]),
                "col16_bound": bool(out[3])}

    def bind(self):
        """Allocate the device workspace (one uint8 tensor) and upload the mesh."""
        if self.ws is not None:
            return self
        self.ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        self._check(self.lib.ns_ctx_bind(self.h, _ptr(self.ws), self.workspace_bytes, _stream_handle(self.device)))
        return self

    def close(self):
        if getattr(self, "h", None):
            self.lib.ns_ctx_destroy(self.h)
            self.h = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, shape=None):
        t = torch.as_tensor(a, dtype=torch.float64, device=self.device)
        if shape is not None:
            t = t.reshape(shape)
        return t.contiguous()

    # ------------------------------------------------------------------ symbolic (host) views
    def pattern(self):
        rp = np.zeros(self.N + 1, np.int32)
        col = np.zeros(self.nnzb, np.int32)
        self._check(self.lib.ns_export_pattern(self.h, rp.ctypes.data_as(_lib.PI), col.ctypes.data_as(_lib.PI)))
        return rp, col

    def fixed_width_offsets(self):
        """[N, w] column offsets (col - row) of the fixed-width rows, 0 past each row's end."""
        w = self.layout()["ell"]
        out = np.zeros(self.N * w, np.int16)
        self._check(self.lib.ns_export_fixed_width_offsets(self.h, out.ctypes.data_as(C.POINTER(C.c_int16))))
        return out.reshape(self.N, w)

    def aggregates(self, level):
        n = self.N
        for lev in range(level):
            n = int(self.aggregates(lev).max()) + 1
        agg = np.zeros(n, np.int32)
        self._check(self.lib.ns_export_aggregates(self.h, level, agg.ctypes.data_as(_lib.PI)))
        return agg

    def colors(self):
        col = np.zeros(len(self._tets), np.int32)
        self._check(self.lib.ns_export_colors(self.h, col.ctypes.data_as(_lib.PI)))
        return col

    # ------------------------------------------------------------------ device work
    def outlet_flow(self, v):
        v = self._dev(v, (self.N, 3))
        out = np.zeros(max(1, self.n_out))
        self._check(self.lib.ns_outlet_flow(self.h, _ptr(v), out.ctypes.data_as(_lib.PD),
                                            _stream_handle(self.device)))
        return out[:self.n_out]

    def rank_one_dots(self, xv):
        xv = self._dev(xv).reshape(-1)[:3 * self.N].contiguous()
        out = np.zeros(max(1, self.n_out))
        self._check(self.lib.ns_rank_one_dots(self.h, _ptr(xv), out.ctypes.data_as(_lib.PD),
                                              _stream_handle(self.device)))
        return out[:self.n_out]

    def _outlet_array(self, a, what):
        if a is None:
            return None
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (self.n_out,)))
        return a

    def assemble(self, v, p, vdot, *, rho, mu, dt, rho_inf, R=None, P_n=None, Q=None, m=None, P_af=None,
                 beta_bf=0.2, c_t=4.0, c_i=36.0, rhs=None):
        """Residual and tangent (Sec. 2.5); returns rhs = -[R_m; R_p] (device, [4N]).

        Outlets: resistances ``R`` (with ``P_n`` and ``Q`` optional, see
        ``ns_phys``: the library forms m^k and P^k_{n+af}), or the reduced
        model's ``m`` and ``P_af`` directly."""
        self.bind()
        v = self._dev(v, (self.N, 3))
        p = self._dev(p, (self.N,))
        vdot = self._dev(vdot, (self.N, 3))
        arrs = {k: self._outlet_array(a, k) for k, a in (("R", R), ("P_n", P_n), ("Q", Q), ("m", m), ("P_af", P_af))}
        if self.n_out and arrs["R"] is None:
            arrs["m"] = arrs["m"] if arrs["m"] is not None else np.zeros(self.n_out)
            arrs["P_af"] = arrs["P_af"] if arrs["P_af"] is not None else np.zeros(self.n_out)
        ptr = {k: (a.ctypes.data_as(_lib.PD) if a is not None else None) for k, a in arrs.items()}
        ph = _lib.NsPhys(rho, mu, dt, rho_inf, beta_bf, c_t, c_i, ptr["m"], ptr["P_af"], ptr["R"], ptr["P_n"],
                         ptr["Q"])
        if rhs is None:
            rhs = torch.empty(4 * self.N, dtype=torch.float64, device=self.device)
        self._check(self.lib.ns_assemble_tangent(self.h, C.byref(ph), _ptr(v), _ptr(p), _ptr(vdot), _ptr(rhs),
                                                 _stream_handle(self.device)))
        self._keep = (v, p, vdot, arrs)  # inputs stay alive until the stream has consumed them
        return rhs

    def resistance_gradient(self, lam, x):
        """dL/dR_k of the last resistance-outlet assembly (``ns_resistance_gradient``),
        from the adjoint solution ``lam`` and the solve's ``x``."""
        lam = self._dev(lam).reshape(-1)
        x = self._dev(x).reshape(-1)
        out = np.zeros(max(1, self.n_out))
        self._check(self.lib.ns_resistance_gradient(self.h, _ptr(lam), _ptr(x), out.ctypes.data_as(_lib.PD),
                                                    _stream_handle(self.device)))
        return out[:self.n_out]

    def _solve(self, fn, b, opts: SolveOptions | None, x=None):
        opts = opts or SolveOptions()
        b = self._dev(b).reshape(-1)
        if b.numel() != 4 * self.N:
            raise ValueError("rhs must have 4N entries")
        if x is None:
            x = torch.empty_like(b)
        co, keep, out = opts.to_c()
        stats = _lib.NsStats()
        st = self._check(fn(self.h, C.byref(co), _ptr(b), _ptr(x), C.byref(stats), _stream_handle(self.device)))
        info = stats.as_dict()
        info["status"] = _lib.STATUS_NAMES[st]
        info["converged"] = st == 0
        if out is not None:
            info["schedule"] = out[:stats.n_calls].tolist()
        return x, info

    def solve(self, rhs, opts: SolveOptions | None = None, x=None):
        """Nested FGMRES + P_SCR solve of the last assembled tangent."""
        return self._solve(self.lib.ns_nested_solve, rhs, opts, x)

    def adjoint(self, g, opts: SolveOptions | None = None, x=None):
        """Solve the transposed system with the transposed nested preconditioner."""
        return self._solve(self.lib.ns_adjoint_solve, g, opts, x)

    def newton_update(self, gamma_dt, dx, y, ydot):
        self._check(self.lib.ns_newton_update(self.h, float(gamma_dt), _ptr(dx), _ptr(y), _ptr(ydot),
                                              _stream_handle(self.device)))

    def time_step(self, y_n, ydot_n, *, rho, mu, dt, rho_inf, model=None, newton=None,
                  opts: SolveOptions | None = None, beta_bf=0.2, c_t=4.0, c_i=36.0):
        """One time step by the predictor multi-corrector algorithm (``ns_time_step``).

        y_n, ydot_n: [4N] field-split state at t_n.  ``model``: dict of per-outlet
        arrays Rp, C, Rd, Pd (P_d at t_{n+1}), Pi, P, Q (values at t_n) and n_ts;
        C = 0 gives the resistance outlet (Rp + Rd) Q + Pd.  ``newton``: dict
        with tol_R, tol_A, eps_abs, eps_rel, l_max.  Returns (y, ydot, stats,
        model') with model' holding Pi, P, Q at t_{n+1}."""
        opts = opts or SolveOptions()
        y_n = self._dev(y_n).reshape(-1)
        ydot_n = self._dev(ydot_n).reshape(-1)
        if y_n.numel() != 4 * self.N or ydot_n.numel() != 4 * self.N:
            raise ValueError("states must have 4N entries")
        y = torch.empty_like(y_n)
        ydot = torch.empty_like(ydot_n)
        no = self.n_out
        model = dict(model or {})
        arrs = {}
        for k, dflt in (("Rp", 0.0), ("C", 0.0), ("Rd", 0.0), ("Pd", 0.0), ("Pi", 0.0), ("P", 0.0), ("Q", 0.0)):
            a = np.ascontiguousarray(np.broadcast_to(np.asarray(model.get(k, dflt), dtype=np.float64), (no,)))
            arrs[k] = a.copy()
        om = _lib.NsOutletModel(*(arrs[k].ctypes.data_as(_lib.PD) for k in ("Rp", "C", "Rd", "Pd", "Pi", "P", "Q")),
                                int(model.get("n_ts", 100)), 0)
        nw = dict(newton or {})
        nopt = _lib.NsNewtonOpts(nw.get("tol_R", 0.0), nw.get("tol_A", 0.0), nw.get("eps_abs", 0.0),
                                 nw.get("eps_rel", 0.0), int(nw.get("l_max", 0)), 0)
        ph = _lib.NsPhys(rho, mu, dt, rho_inf, beta_bf, c_t, c_i, None, None)
        co, keep, _ = opts.to_c()
        stats = _lib.NsStepStats()
        st = self._check(self.lib.ns_time_step(self.h, C.byref(ph), C.byref(om), C.byref(nopt), C.byref(co),
                                               _ptr(y_n), _ptr(ydot_n), _ptr(y), _ptr(ydot), C.byref(stats),
                                               _stream_handle(self.device)))
        info = stats.as_dict()
        info["status"] = _lib.STATUS_NAMES[st]
        out = {k: arrs[k] for k in ("Pi", "P", "Q")}
        return y, ydot, info, out

    def kernel_timing(self, classes=(), period: int = 1):
        """Time launches of the given kernel classes (see ``ns_kernel_class``) in later solves,
        every ``period``-th launch of each class."""
        mask = 0
        for k in classes:
            mask |= 1 << _lib.KERNEL_CLASSES[k]
        self._check(self.lib.ns_kernel_timing_period(self.h, int(period)))
        self._check(self.lib.ns_kernel_timing(self.h, mask))

    def kernel_timing_read(self, cls):
        """(launches, total ms, algorithmic bytes) of a kernel class since the last read."""
        out = (C.c_double * 3)()
        self._check(self.lib.ns_kernel_timing_read(self.h, _lib.KERNEL_CLASSES[cls], out))
        return int(out[0]), float(out[1]), float(out[2])

    def export_bsr(self, transposed=False):
        out = torch.empty((self.nnzb, 4, 4), dtype=torch.float64, device=self.device)
        self._check(self.lib.ns_export_bsr(self.h, int(transposed), _ptr(out), _stream_handle(self.device)))
        return out

    def export_shat(self):
        nS = self.sizes[2]
        rp = np.zeros(self.N + 1, np.int32)
        col = np.zeros(nS, np.int32)
        val = torch.empty(nS, dtype=torch.float64, device=self.device)
        self._check(self.lib.ns_export_shat(self.h, rp.ctypes.data_as(_lib.PI), col.ctypes.data_as(_lib.PI),
                                            _ptr(val), _stream_handle(self.device)))
        return rp, col, val

    def outlet_vectors(self):
        out = torch.empty((max(1, self.n_out), self.N, 3), dtype=torch.float64, device=self.device)
        self._check(self.lib.ns_export_outlet_vectors(self.h, _ptr(out), _stream_handle(self.device)))
        return out[:self.n_out]

    def apply(self, op: str, x, opts: SolveOptions | None = None):
        """One operator of the forward system (see ``ns_op``); returns (y, schedule)."""
        sizes_in = {"full": 4, "A": 3, "B": 1, "C": 3, "D": 1, "shat": 1, "vcycle_A": 3, "vcycle_S": 1,
                    "schur": 1, "pscr": 4, "solve_A": 3, "psimple": 4}
        sizes_out = {"full": 4, "A": 3, "B": 3, "C": 1, "D": 1, "shat": 1, "vcycle_A": 3, "vcycle_S": 1,
                     "schur": 1, "pscr": 4, "solve_A": 3, "psimple": 4}
        x = self._dev(x).reshape(-1)
        if x.numel() != sizes_in[op] * self.N:
            raise ValueError(f"operator {op} takes {sizes_in[op]}N entries")
        y = torch.empty(sizes_out[op] * self.N, dtype=torch.float64, device=self.device)
        opts = opts or SolveOptions()
        co, keep, out = opts.to_c()
        self._check(self.lib.ns_apply(self.h, _lib.OPS[op], C.byref(co), _ptr(x), _ptr(y),
                                      _stream_handle(self.device)))
        return y, out


def stream_bench(mode: int, src: torch.Tensor, dst: torch.Tensor, reps: int = 10) -> float:
    """Average ms per launch of the streaming kernel ``mode`` (0 read, 1 copy)
    over src.numel() bytes (``ns_stream_bench``); src and dst are device byte tensors."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst smaller than src")
    out = C.c_double()
    with torch.cuda.device(src.device):
        torch.cuda.synchronize()
        st = _lib.load().ns_stream_bench(int(mode), _ptr(src), _ptr(dst), nbytes, int(reps), C.byref(out))
    if st != 0:
        raise NsError(st, "ns_stream_bench failed")
    return out.value


def context_for(case, **kw) -> NsContext:
    return NsContext(case, **kw).bind()


def gen_alpha(rho_inf):
    """(alpha_m, alpha_f, gamma) of the generalized-alpha method (``ns_gen_alpha``)."""
    out = (C.c_double * 3)()
    st = _lib.load().ns_gen_alpha(float(rho_inf), out)
    if st != 0:
        raise NsError(st, "rho_inf must lie in [0, 1]")
    return out[0], out[1], out[2]


class NestedSolveFn(torch.autograd.Function):
    """x(R) = A(R)^{-1} r(R) for one Newton step at a frozen state, with
    resistance outlets: the library forms m^k = R^k and
    P^k_{n+af} = (1 - alpha_f) P^k_n + alpha_f R^k Q^k (``ns_phys.h_R``), and
    backward solves A^T lam = dL/dx with the transposed nested preconditioner
    (``ns_adjoint_solve``) and contracts dL/dR on the device
    (``ns_resistance_gradient``).

    apply(R, ctx, case, P_n, Q, fwd_opts, adj_opts) -> x  (R: CPU float64 [n_out])
    """

    @staticmethod
    def forward(fctx, R, ctx: NsContext, case, P_n, Q, fwd_opts=None, adj_opts=None):
        rhs = ctx.assemble(case.v, case.p, case.vdot, rho=case.rho, mu=case.mu, dt=case.dt,
                           rho_inf=case.rho_inf, R=R.detach().cpu().double().numpy(), P_n=P_n, Q=Q)
        x, info = ctx.solve(rhs, fwd_opts)
        fctx.ctx = ctx
        fctx.adj_opts = adj_opts
        fctx.info = info
        fctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(fctx, grad_x):
        (x,) = fctx.saved_tensors
        ctx = fctx.ctx
        lam, info = ctx.adjoint(grad_x.contiguous(), fctx.adj_opts)
        grad_R = ctx.resistance_gradient(lam, x)
        return (torch.as_tensor(grad_R, dtype=torch.float64), None, None, None, None, None, None)
