"""Thin ctypes binding over the C-ABI of libgnmpc.so (include/gnmpc.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  Device arrays are torch tensors on the plan's GPU (torch provides the
memory and the stream); host arrays are numpy arrays.  There is no fallback:
if the library is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # loads torch's HIP runtime first, so the library binds to the same one

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgnmpc.so")

OK, INVALID_ARG, BAD_GRAPH, SHAPE, UNSUPPORTED, HIP_ERROR, BAD_CONSTRAINT, NOT_READY, NO_DEVICE = range(9)
F64, F32, BF16 = 0, 1, 2
QP_SOLVED, QP_MAXITER, QP_PRIMAL_INFEASIBLE, QP_NONFINITE, QP_NOT_PD = range(5)
LIN_FINITE, LIN_NONFINITE_INPUT, LIN_NONFINITE_OUTPUT = range(3)
LIN_ARRAYS = ("xhat", "uhat", "A", "B", "c", "fnext")
PHASES = ("gnn_forward", "gnn_jacobian", "gnn_assembly", "msd_linearize", "condense_propagate",
          "condense_gram", "condense_rows", "qp", "gnn_stage_images")


class GnmpcError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"gnmpc status {status} ({status_string(status)}): {msg}")


class Dims(C.Structure):
    _fields_ = [("M", C.c_int32), ("nu", C.c_int32), ("N", C.c_int32), ("n_c_max", C.c_int32),
                ("dtype", C.c_int32)]


class MsdParams(C.Structure):
    _fields_ = [("k", C.c_double), ("c", C.c_double), ("m", C.c_double), ("dt", C.c_double),
                ("k3", C.c_double), ("gravity", C.c_double), ("anchor", C.c_int32), ("reserved", C.c_int32)]


class GnnDesc(C.Structure):
    _fields_ = [("Hd", C.c_int32), ("L", C.c_int32), ("dtype", C.c_int32), ("reserved", C.c_int32),
                ("dt", C.c_double)]


class InetDesc(C.Structure):
    _fields_ = [("psi_hidden", C.c_int32), ("psi_width", C.c_int32), ("d_m", C.c_int32),
                ("phi_hidden", C.c_int32), ("phi_width", C.c_int32), ("nu", C.c_int32), ("dt", C.c_double)]


class TuneEntry(C.Structure):
    _fields_ = [("variant", C.c_int32), ("block_nodes", C.c_int32), ("us", C.c_double)]


class TuneReport(C.Structure):
    _fields_ = [("count", C.c_int32), ("chosen", C.c_int32), ("entry", TuneEntry * 16)]


class AdmmSettings(C.Structure):
    _fields_ = [("rho", C.c_double), ("sigma", C.c_double), ("alpha", C.c_double), ("eps_abs", C.c_double),
                ("eps_rel", C.c_double), ("kappa_fp64", C.c_double), ("max_iter", C.c_int32),
                ("check_every", C.c_int32)]


class QpInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("used_fp64", C.c_int32), ("reserved", C.c_int32),
                ("prim_res", C.c_double), ("dual_res", C.c_double), ("kappa_est", C.c_double), ("obj", C.c_double)]


QP_INFO_BYTES = C.sizeof(QpInfo)


class LinInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("first_array", C.c_int32), ("first_stage", C.c_int32),
                ("first_node", C.c_int32), ("nonfinite", C.c_int64 * 6)]


LIN_INFO_BYTES = C.sizeof(LinInfo)


class StepDesc(C.Structure):
    _fields_ = [("plan", C.c_void_p)] + [(f, C.c_void_p) for f in (
        "xhat", "uhat", "x0", "Q", "q", "R", "r", "rowC", "rowd", "lb", "ub", "lc", "uc")] + [
        ("Q_full", C.c_int32), ("reserved", C.c_int32)] + [(f, C.c_void_p) for f in (
        "A", "B", "c", "H", "g", "Ct", "dt", "u")] + [("info", C.c_void_p)]

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} not found: build it with `python -m paper_2602_17601_amd.build_lib`")
        L = C.CDLL(_LIB_PATH)
        i32, i64, vp = C.c_int32, C.c_int64, C.c_void_p
        P = C.POINTER
        sig = {
            "gnmpc_version": ([], C.c_char_p),
            "gnmpc_status_string": ([i32], C.c_char_p),
            "gnmpc_graph_check": ([vp, vp, i32, i32], i32),
            "gnmpc_graph_closure": ([vp, vp, i32, i32, i32, vp, vp, i64, P(i64)], i32),
            "gnmpc_plan_create": ([P(vp), P(Dims), i32], i32),
            "gnmpc_plan_destroy": ([vp], None),
            "gnmpc_plan_last_error": ([vp], C.c_char_p),
            "gnmpc_graph_set": ([vp, vp, vp, i32, i32, i32], i32),
            "gnmpc_graph_nnz": ([vp, P(i64)], i32),
            "gnmpc_graph_pattern": ([vp, vp, vp], i32),
            "gnmpc_model_set_msd": ([vp, P(MsdParams), vp, i32], i32),
            "gnmpc_model_set_gnn": ([vp, P(GnnDesc), vp, i64, vp, i32], i32),
            "gnmpc_model_set_inet": ([vp, P(InetDesc), vp, i64], i32),
            "gnmpc_rows_set": ([vp, i32, vp, vp], i32),
            "gnmpc_linearize": ([vp] + [vp] * 8, i32),
            "gnmpc_rollout_linear": ([vp] * 8, i32),
            "gnmpc_jvp": ([vp] * 7, i32),
            "gnmpc_vjp": ([vp] * 7, i32),
            "gnmpc_condense": ([vp, vp, vp, vp, vp, vp, i32] + [vp] * 11, i32),
            "gnmpc_condense_variant_set": ([vp, i32, i32], i32),
            "gnmpc_condense_variant_get": ([vp, P(i32), P(i32)], i32),
            "gnmpc_autotune_condense": ([vp, vp, vp, vp, vp, vp, i32] + [vp] * 9 + [i32, P(TuneReport), vp], i32),
            "gnmpc_solve_box_qp": ([vp, i32, vp, vp, vp, vp, i32, vp, vp, vp, P(AdmmSettings), vp, vp, vp], i32),
            "gnmpc_gnn_forward": ([vp, vp, vp, vp, vp], i32),
            "gnmpc_msd_simulate": ([vp, i32, i32, vp, vp, vp, vp], i32),
            "gnmpc_gnn_vjp": ([vp, vp, vp, vp, vp, vp, vp], i32),
            "gnmpc_gnn_train_sizes": ([vp, P(i64), P(i64)], i32),
            "gnmpc_gnn_loss_grad": ([vp, vp, vp, vp, vp, vp, C.c_double, vp, vp, vp, vp], i32),
            "gnmpc_adam_step": ([i64, vp, vp, vp, vp, i32, C.c_double, C.c_double, C.c_double, C.c_double, vp], i32),
            "gnmpc_solve_qp_ipm": ([vp, i32, vp, vp, vp, vp, i32, vp, vp, vp, C.c_double, i32, vp, vp, vp], i32),
            "gnmpc_solve_box_qp_noalloc": ([i32, i32, vp, vp, vp, vp, i32, vp, vp, vp, P(AdmmSettings), vp, vp, vp],
                                           i32),
            "gnmpc_admm_default_settings": ([P(AdmmSettings)], None),
            "gnmpc_timers_enable": ([vp, i32], i32),
            "gnmpc_step_batched": ([vp, i32, P(AdmmSettings), vp], i32),
            "gnmpc_rti_step": ([P(StepDesc), vp, vp, vp, P(AdmmSettings), vp], i32),
            "gnmpc_rti_step_ipm": ([P(StepDesc), vp, vp, vp, C.c_double, i32, vp], i32),
            "gnmpc_timers_read": ([vp, vp, vp], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def status_string(s):
    try:
        return lib().gnmpc_status_string(int(s)).decode()
    except ImportError:
        return "?"


def version():
    return lib().gnmpc_version().decode()


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _hp(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None and a.size else None


def graph_check(row_ptr, col):
    rp, cl = _i32(row_ptr), _i32(col)
    return lib().gnmpc_graph_check(_hp(rp), _hp(cl), len(rp) - 1, len(cl))


def graph_closure(row_ptr, col, L):
    """Jacobian block pattern (row_ptr, col) of the L-round closure (host)."""
    rp, cl = _i32(row_ptr), _i32(col)
    M = len(rp) - 1
    nnz = C.c_int64(0)
    s = lib().gnmpc_graph_closure(_hp(rp), _hp(cl), M, len(cl), L, None, None, 0, C.byref(nnz))
    if s != OK:
        raise GnmpcError(s, "graph_closure")
    prow = np.zeros(M + 1, np.int32)
    pcol = np.zeros(nnz.value, np.int32)
    s = lib().gnmpc_graph_closure(_hp(rp), _hp(cl), M, len(cl), L, _hp(prow), _hp(pcol), nnz.value, C.byref(nnz))
    if s != OK:
        raise GnmpcError(s, "graph_closure")
    return prow, pcol


def default_admm_settings(**kw):
    s = AdmmSettings()
    lib().gnmpc_admm_default_settings(C.byref(s))
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Plan:
    """A gnmpc plan: dimensions, graph, model, state rows and all workspace."""

    def __init__(self, M, nu, N, n_c_max=0, dtype=F32, device=0):
        self.M, self.nu, self.N, self.n_c_max, self.dtype = M, nu, N, n_c_max, dtype
        self.device = device
        self.tdtype = torch.float64 if dtype == F64 else torch.float32
        d = Dims(M, nu, N, n_c_max, dtype)
        h = C.c_void_p()
        s = lib().gnmpc_plan_create(C.byref(h), C.byref(d), device)
        if s != OK:
            raise GnmpcError(s, "plan_create")
        self._h = h
        self.nnz = None
        self.n_c = 0

    def close(self):
        if getattr(self, "_h", None):
            lib().gnmpc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s, what):
        if s != OK:
            msg = lib().gnmpc_plan_last_error(self._h).decode()
            raise GnmpcError(s, f"{what}: {msg}")

    def _dev(self, t, shape, name, dtype=None, allow_none=False):
        if t is None:
            if allow_none:
                return None
            raise GnmpcError(INVALID_ARG, f"{name} is required")
        dtype = dtype or self.tdtype
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.device.index == self.device):
            raise GnmpcError(INVALID_ARG, f"{name} must be a tensor on cuda:{self.device}")
        if t.dtype != dtype or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise GnmpcError(SHAPE, f"{name}: expected contiguous {dtype} {tuple(shape)}, got {t.dtype} "
                                    f"{tuple(t.shape)} contiguous={t.is_contiguous()}")
        return C.c_void_p(t.data_ptr())

    # ---- setup
    def graph_set(self, row_ptr, col, L):
        rp, cl = _i32(row_ptr), _i32(col)
        self._check(lib().gnmpc_graph_set(self._h, _hp(rp), _hp(cl), len(rp) - 1, len(cl), L), "graph_set")
        n = C.c_int64(0)
        self._check(lib().gnmpc_graph_nnz(self._h, C.byref(n)), "graph_nnz")
        self.nnz = n.value
        self.L = L

    def graph_pattern(self):
        prow = np.zeros(self.M + 1, np.int32)
        pcol = np.zeros(self.nnz, np.int32)
        self._check(lib().gnmpc_graph_pattern(self._h, _hp(prow), _hp(pcol)), "graph_pattern")
        return prow, pcol

    def model_set_msd(self, prm, act):
        p = MsdParams(prm.k, prm.c, prm.m, prm.dt, prm.k3, prm.gravity, prm.anchor, 0)
        a = _i32(act)
        self._check(lib().gnmpc_model_set_msd(self._h, C.byref(p), _hp(a), len(a)), "model_set_msd")
        self.model = "msd"

    def gnn_train_sizes(self):
        """(number of parameters, workspace bytes) of gnmpc_gnn_loss_grad."""
        n, b = C.c_int64(), C.c_int64()
        self._check(lib().gnmpc_gnn_train_sizes(self._h, C.byref(n), C.byref(b)), "gnn_train_sizes")
        return n.value, b.value

    def gnn_loss_grad(self, theta, x, u, x_next, O, lam, workspace, loss, grad, stream=None):
        """gnmpc_gnn_loss_grad over the plan's N samples: loss [1] and grad [n_params]
        (FP32 device) at theta (FP32 device, the packing of gnn_flat)."""
        M, N, nu = self.M, self.N, self.nu
        n, wb = self.gnn_train_sizes()
        Oh = np.ascontiguousarray(np.asarray(O, dtype=np.float32).reshape(6))
        args = [self._dev(theta, (n,), "theta", dtype=torch.float32), self._dev(x, (N, M, 6), "x"),
                self._dev(u, (N, nu), "u"), self._dev(x_next, (N, M, 6), "x_next"), _hp(Oh), float(lam),
                self._dev(workspace, (wb,), "workspace", dtype=torch.uint8),
                self._dev(loss, (1,), "loss", dtype=torch.float32), self._dev(grad, (n,), "grad", dtype=torch.float32)]
        self._check(lib().gnmpc_gnn_loss_grad(self._h, *args, _stream(stream)), "gnn_loss_grad")

    def model_set_inet(self, W):
        """The interaction network (workloads.InetWeights) as the plan's model."""
        d = InetDesc(len(W.psi_W) - 1, int(W.psi_W[0].shape[0]) if len(W.psi_W) > 1 else 1, W.d_m,
                     len(W.phi_W) - 1, int(W.phi_W[0].shape[0]) if len(W.phi_W) > 1 else 1, W.nu, W.dt)
        flat = np.ascontiguousarray(W.flat(), dtype=np.float64)
        self._check(lib().gnmpc_model_set_inet(self._h, C.byref(d), _hp(flat), flat.shape[0]), "model_set_inet")
        self.model = "inet"

    def model_set_gnn(self, W, act, dtype=F32):
        w = gnn_flat(W)
        d = GnnDesc(W.Hd, W.L, dtype, 0, W.dt)
        a = _i32(act)
        self._check(lib().gnmpc_model_set_gnn(self._h, C.byref(d), _hp(w), w.size, _hp(a), len(a)),
                    "model_set_gnn")
        self.model = "gnn"

    def rows_set(self, node, stage):
        n, st = _i32(node), _i32(stage)
        self._check(lib().gnmpc_rows_set(self._h, len(n), _hp(n), _hp(st)), "rows_set")
        self.n_c = len(n)

    # ---- hot path
    def linearize(self, xhat, uhat, A, B, c, fnext=None, info=None, stream=None):
        """A, B, c (and fnext) at the N points (gnmpc_linearize); info, a uint8 tensor of
        LIN_INFO_BYTES on the device, receives the finiteness report (decode with lin_info)."""
        M, N, nu = self.M, self.N, self.nu
        args = [self._dev(xhat, (N + 1, M, 6), "xhat"), self._dev(uhat, (N, nu), "uhat"),
                self._dev(A, (N, self.nnz, 6, 6), "A"), self._dev(B, (N, M, 6, nu), "B"),
                self._dev(c, (N, M, 6), "c"), self._dev(fnext, (N, M, 6), "fnext", allow_none=True),
                self._dev(info, (LIN_INFO_BYTES,), "info", dtype=torch.uint8, allow_none=True)]
        self._check(lib().gnmpc_linearize(self._h, *args, _stream(stream)), "linearize")

    def rollout_linear(self, A, B, c, x0, u, x, stream=None):
        """x[0] = x0, x[k+1] = A_k x[k] + B_k u[k] + c_k (gnmpc_rollout_linear)."""
        M, N, nu = self.M, self.N, self.nu
        args = [self._dev(A, (N, self.nnz, 6, 6), "A"), self._dev(B, (N, M, 6, nu), "B"),
                self._dev(c, (N, M, 6), "c"), self._dev(x0, (M, 6), "x0"), self._dev(u, (N, nu), "u"),
                self._dev(x, (N + 1, M, 6), "x")]
        self._check(lib().gnmpc_rollout_linear(self._h, *args, _stream(stream)), "rollout_linear")

    def msd_simulate(self, x0, u, X, stream=None):
        """X[b][0] = x0[b], X[b][t+1] = f(X[b][t], u[b][t]) with the plan's spring-damper
        model (gnmpc_msd_simulate); x0 [B][M][6], u [B][T][nu], X [B][T+1][M][6]."""
        B, T = X.shape[0], X.shape[1] - 1
        args = [self._dev(x0, (B, self.M, 6), "x0"), self._dev(u, (B, T, self.nu), "u"),
                self._dev(X, (B, T + 1, self.M, 6), "X")]
        self._check(lib().gnmpc_msd_simulate(self._h, B, T, *args, _stream(stream)), "msd_simulate")

    def gnn_forward(self, xhat, uhat, fnext, stream=None):
        """fnext[k] = f(xhat[k], uhat[k]) with the plan's GNN (gnmpc_gnn_forward)."""
        M, N, nu = self.M, self.N, self.nu
        args = [self._dev(xhat, (N + 1, M, 6), "xhat"), self._dev(uhat, (N, nu), "uhat"),
                self._dev(fnext, (N, M, 6), "fnext")]
        self._check(lib().gnmpc_gnn_forward(self._h, *args, _stream(stream)), "gnn_forward")

    def gnn_vjp(self, xhat, uhat, g, gx, gu, stream=None):
        """gx[k] = (df/dx_k)' g[k], gu[k] = (df/du_k)' g[k] by reverse mode through the
        GNN's layers (gnmpc_gnn_vjp)."""
        M, N, nu = self.M, self.N, self.nu
        args = [self._dev(xhat, (N + 1, M, 6), "xhat"), self._dev(uhat, (N, nu), "uhat"),
                self._dev(g, (N, M, 6), "g"), self._dev(gx, (N, M, 6), "gx"), self._dev(gu, (N, nu), "gu")]
        self._check(lib().gnmpc_gnn_vjp(self._h, *args, _stream(stream)), "gnn_vjp")

    def jvp(self, A, B, dx, du, out, stream=None):
        """out[k] = A_k dx[k] + B_k du[k] (gnmpc_jvp)."""
        M, N, nu = self.M, self.N, self.nu
        args = [self._dev(A, (N, self.nnz, 6, 6), "A"), self._dev(B, (N, M, 6, nu), "B"),
                self._dev(dx, (N, M, 6), "dx"), self._dev(du, (N, nu), "du"), self._dev(out, (N, M, 6), "out")]
        self._check(lib().gnmpc_jvp(self._h, *args, _stream(stream)), "jvp")

    def vjp(self, A, B, g, gx, gu, stream=None):
        """gx[k] = A_k' g[k], gu[k] = B_k' g[k] (gnmpc_vjp)."""
        M, N, nu = self.M, self.N, self.nu
        args = [self._dev(A, (N, self.nnz, 6, 6), "A"), self._dev(B, (N, M, 6, nu), "B"),
                self._dev(g, (N, M, 6), "g"), self._dev(gx, (N, M, 6), "gx"), self._dev(gu, (N, nu), "gu")]
        self._check(lib().gnmpc_vjp(self._h, *args, _stream(stream)), "vjp")

    def condense(self, A, B, c, x0, Q, q, R, r, rowC, rowd, H, g, Ct, dt, Gx=None, stream=None):
        M, N, nu, nc = self.M, self.N, self.nu, self.n_c
        full = 1 if Q.dim() == 4 else 0
        qshape = (N + 1, M, 6, 6) if full else (N + 1, M, 6)
        n = N * nu
        args = [self._dev(A, (N, self.nnz, 6, 6), "A"), self._dev(B, (N, M, 6, nu), "B"),
                self._dev(c, (N, M, 6), "c"), self._dev(x0, (M, 6), "x0"), self._dev(Q, qshape, "Q"), full,
                self._dev(q, (N + 1, M, 6), "q"), self._dev(R, (N, nu, nu), "R"), self._dev(r, (N, nu), "r"),
                self._dev(rowC, (nc, 6), "rowC", allow_none=nc == 0),
                self._dev(rowd, (nc,), "rowd", allow_none=nc == 0),
                self._dev(H, (n, n), "H"), self._dev(g, (n,), "g"),
                self._dev(Ct, (nc, n), "Ct", allow_none=nc == 0), self._dev(dt, (nc,), "dt", allow_none=nc == 0),
                self._dev(Gx, (N + 1, M, 6), "Gx", allow_none=True)]
        self._check(lib().gnmpc_condense(self._h, *args, _stream(stream)), "condense")

    def autotune_condense(self, A, B, c, x0, Q, q, R, r, rowC, rowd, H, g, Ct, dt, reps=5, stream=None):
        """gnmpc_autotune_condense: time every propagation variant on these arrays, keep
        the fastest; returns (chosen index, [dict(variant, block_nodes, us)])."""
        M, N, nu, nc = self.M, self.N, self.nu, self.n_c
        full = 1 if Q.dim() == 4 else 0
        qshape = (N + 1, M, 6, 6) if full else (N + 1, M, 6)
        n = N * nu
        args = [self._dev(A, (N, self.nnz, 6, 6), "A"), self._dev(B, (N, M, 6, nu), "B"),
                self._dev(c, (N, M, 6), "c"), self._dev(x0, (M, 6), "x0"), self._dev(Q, qshape, "Q"), full,
                self._dev(q, (N + 1, M, 6), "q"), self._dev(R, (N, nu, nu), "R"), self._dev(r, (N, nu), "r"),
                self._dev(rowC, (nc, 6), "rowC", allow_none=nc == 0), self._dev(rowd, (nc,), "rowd", allow_none=nc == 0),
                self._dev(H, (n, n), "H"), self._dev(g, (n,), "g"),
                self._dev(Ct, (nc, n), "Ct", allow_none=nc == 0), self._dev(dt, (nc,), "dt", allow_none=nc == 0)]
        rep = TuneReport()
        self._check(lib().gnmpc_autotune_condense(self._h, *args, int(reps), C.byref(rep), _stream(stream)),
                    "autotune_condense")
        return rep.chosen, [dict(variant=rep.entry[t].variant, block_nodes=rep.entry[t].block_nodes, us=rep.entry[t].us)
                            for t in range(rep.count)]

    def condense_variant(self, variant=None, block_nodes=0):
        """Set the propagation variant (gnmpc_condense_variant_set) when given; return
        the current (variant, block_nodes)."""
        if variant is not None:
            self._check(lib().gnmpc_condense_variant_set(self._h, int(variant), int(block_nodes)), "condense_variant")
        v, nb = C.c_int32(), C.c_int32()
        self._check(lib().gnmpc_condense_variant_get(self._h, C.byref(v), C.byref(nb)), "condense_variant")
        return v.value, nb.value

    def solve_qp_ipm(self, H, g, lb, ub, Ct, lc, uc, u, info=None, tol=1e-9, max_iter=100, stream=None):
        """gnmpc_solve_qp_ipm: the same QP by the interior-point method."""
        n = g.shape[0]
        nc = 0 if Ct is None else Ct.shape[0]
        args = [self._dev(H, (n, n), "H"), self._dev(g, (n,), "g"), self._dev(lb, (n,), "lb"),
                self._dev(ub, (n,), "ub"), nc, self._dev(Ct, (nc, n), "Ct", allow_none=nc == 0),
                self._dev(lc, (nc,), "lc", allow_none=True), self._dev(uc, (nc,), "uc", allow_none=True),
                float(tol), int(max_iter), self._dev(u, (n,), "u"),
                self._dev(info, (QP_INFO_BYTES,), "info", dtype=torch.uint8, allow_none=True)]
        self._check(lib().gnmpc_solve_qp_ipm(self._h, n, *args, _stream(stream)), "solve_qp_ipm")

    def solve_box_qp(self, H, g, lb, ub, Ct, lc, uc, u, info=None, settings=None, stream=None):
        n = g.shape[0]
        nc = 0 if Ct is None else Ct.shape[0]
        st = settings or default_admm_settings()
        args = [self._dev(H, (n, n), "H"), self._dev(g, (n,), "g"), self._dev(lb, (n,), "lb"),
                self._dev(ub, (n,), "ub"), nc, self._dev(Ct, (nc, n), "Ct", allow_none=nc == 0),
                self._dev(lc, (nc,), "lc", allow_none=True), self._dev(uc, (nc,), "uc", allow_none=True),
                C.byref(st), self._dev(u, (n,), "u"),
                self._dev(info, (QP_INFO_BYTES,), "info", dtype=torch.uint8, allow_none=True)]
        self._check(lib().gnmpc_solve_box_qp(self._h, n, *args, _stream(stream)), "solve_box_qp")


def _timers_enable(self, on=True):
    self._check(lib().gnmpc_timers_enable(self._h, 1 if on else 0), "timers_enable")


def _timers_read(self):
    """{phase: (total_ms, count)} for the records since timers were enabled (synchronizes)."""
    tot = np.zeros(len(PHASES), np.float64)
    cnt = np.zeros(len(PHASES), np.int32)
    self._check(lib().gnmpc_timers_read(self._h, _hp(tot), _hp(cnt)), "timers_read")
    return {name: (float(tot[i]), int(cnt[i])) for i, name in enumerate(PHASES)}


Plan.timers_enable = _timers_enable
Plan.timers_read = _timers_read


def solve_box_qp_noalloc(H, g, lb, ub, Ct, lc, uc, u, info=None, settings=None, stream=None):
    """gnmpc_solve_box_qp_noalloc: the box QP with no plan and no allocation
    (workspace in the library's static per-GPU array; n <= 464).  All tensors
    on the current device, float32 or float64 (the dtype of H)."""
    dtype = H.dtype
    if dtype not in (torch.float32, torch.float64):
        raise GnmpcError(INVALID_ARG, "solve_box_qp_noalloc: float32 or float64 arrays")
    dev = torch.cuda.current_device()
    n = g.shape[0]
    nc = 0 if Ct is None else Ct.shape[0]

    def arg(t, shape, name, dt=dtype, allow_none=False):
        if t is None:
            if allow_none:
                return None
            raise GnmpcError(INVALID_ARG, f"{name} is required")
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.device.index == dev):
            raise GnmpcError(INVALID_ARG, f"{name} must be a tensor on cuda:{dev}")
        if t.dtype != dt or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise GnmpcError(SHAPE, f"{name}: expected contiguous {dt} {tuple(shape)}, got {t.dtype} "
                                    f"{tuple(t.shape)} contiguous={t.is_contiguous()}")
        return C.c_void_p(t.data_ptr())

    st = settings or default_admm_settings()
    args = [arg(H, (n, n), "H"), arg(g, (n,), "g"), arg(lb, (n,), "lb"), arg(ub, (n,), "ub"), nc,
            arg(Ct, (nc, n), "Ct", allow_none=nc == 0), arg(lc, (nc,), "lc", allow_none=True),
            arg(uc, (nc,), "uc", allow_none=True), C.byref(st), arg(u, (n,), "u"),
            arg(info, (QP_INFO_BYTES,), "info", dt=torch.uint8, allow_none=True)]
    s = lib().gnmpc_solve_box_qp_noalloc(F64 if dtype == torch.float64 else F32, n, *args, _stream(stream))
    if s != OK:
        raise GnmpcError(s, "solve_box_qp_noalloc: " + status_string(s))


def gnn_flat(W):
    """The GNN's parameters packed as the library takes them (float64): W_enc, b_enc,
    per round W_e, b_e, W_n, b_n, then W_dec, b_dec."""
    flat = [W.W_enc, W.b_enc]
    for l in range(W.L):
        flat += [W.W_edge[l], W.b_edge[l], W.W_node[l], W.b_node[l]]
    flat += [W.W_dec, W.b_dec]
    return np.ascontiguousarray(np.concatenate([np.asarray(x, np.float64).reshape(-1) for x in flat]))


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """gnmpc_adam_step in place on FP32 device tensors of equal size."""
    n = theta.numel()
    for t, name in ((theta, "theta"), (grad, "grad"), (m, "m"), (v, "v")):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
                and t.numel() == n):
            raise GnmpcError(SHAPE, f"adam_step: {name} must be a contiguous float32 CUDA tensor of {n} entries")
    s = lib().gnmpc_adam_step(n, C.c_void_p(theta.data_ptr()), C.c_void_p(grad.data_ptr()), C.c_void_p(m.data_ptr()),
                              C.c_void_p(v.data_ptr()), int(step), lr, beta1, beta2, eps, _stream(stream))
    if s != OK:
        raise GnmpcError(s, "adam_step")


def step_desc(plan, b):
    """The descriptor of one instance's step: `b` maps xhat, uhat, x0, Q, q, R,
    r, rowC, rowd, lb, ub, (lc, uc), A, B, c, H, g, Ct, dt, u, (info) to tensors
    of the plan's shapes (the same checks as the single calls)."""
    M, N, nu, nc, n = plan.M, plan.N, plan.nu, plan.n_c, plan.N * plan.nu
    full = 1 if b["Q"].dim() == 4 else 0
    d = StepDesc()
    d.plan = plan._h
    dv = plan._dev
    d.xhat, d.uhat = dv(b["xhat"], (N + 1, M, 6), "xhat"), dv(b["uhat"], (N, nu), "uhat")
    d.x0 = dv(b["x0"], (M, 6), "x0")
    d.Q = dv(b["Q"], (N + 1, M, 6, 6) if full else (N + 1, M, 6), "Q")
    d.q, d.R, d.r = dv(b["q"], (N + 1, M, 6), "q"), dv(b["R"], (N, nu, nu), "R"), dv(b["r"], (N, nu), "r")
    d.rowC = dv(b.get("rowC"), (nc, 6), "rowC", allow_none=nc == 0)
    d.rowd = dv(b.get("rowd"), (nc,), "rowd", allow_none=nc == 0)
    d.lb, d.ub = dv(b["lb"], (n,), "lb"), dv(b["ub"], (n,), "ub")
    d.lc = dv(b.get("lc"), (nc,), "lc", allow_none=True)
    d.uc = dv(b.get("uc"), (nc,), "uc", allow_none=True)
    d.Q_full = full
    d.A, d.B = dv(b["A"], (N, plan.nnz, 6, 6), "A"), dv(b["B"], (N, M, 6, nu), "B")
    d.c, d.H, d.g = dv(b["c"], (N, M, 6), "c"), dv(b["H"], (n, n), "H"), dv(b["g"], (n,), "g")
    d.Ct = dv(b.get("Ct"), (nc, n), "Ct", allow_none=nc == 0)
    d.dt = dv(b.get("dt"), (nc,), "dt", allow_none=nc == 0)
    d.u = dv(b["u"], (n,), "u")
    d.info = dv(b.get("info"), (QP_INFO_BYTES,), "info", dtype=torch.uint8, allow_none=True)
    return d


def rti_step(plan, b, xpred, xhat_next=None, uhat_next=None, settings=None, stream=None):
    """gnmpc_rti_step: one iteration of Algorithm 1 on the buffers `b` (as for
    step_desc); x* goes to xpred [N+1][M][6] and the shifted linearization
    trajectory to xhat_next / uhat_next (default: b["xhat"], b["uhat"] in place)."""
    d = step_desc(plan, b)
    xn = b["xhat"] if xhat_next is None else xhat_next
    un = b["uhat"] if uhat_next is None else uhat_next
    M, N, nu = plan.M, plan.N, plan.nu
    args = [plan._dev(xpred, (N + 1, M, 6), "xpred"), plan._dev(xn, (N + 1, M, 6), "xhat_next"),
            plan._dev(un, (N, nu), "uhat_next")]
    st = settings or default_admm_settings()
    plan._check(lib().gnmpc_rti_step(C.byref(d), *args, C.byref(st), _stream(stream)), "rti_step")


def rti_step_ipm(plan, b, xpred, xhat_next=None, uhat_next=None, tol=1e-9, max_iter=100, stream=None):
    """gnmpc_rti_step_ipm: rti_step with the condensed QP solved by the
    interior-point method (tol on the duality measure, max_iter iterations)."""
    d = step_desc(plan, b)
    xn = b["xhat"] if xhat_next is None else xhat_next
    un = b["uhat"] if uhat_next is None else uhat_next
    M, N, nu = plan.M, plan.N, plan.nu
    args = [plan._dev(xpred, (N + 1, M, 6), "xpred"), plan._dev(xn, (N + 1, M, 6), "xhat_next"),
            plan._dev(un, (N, nu), "uhat_next")]
    plan._check(lib().gnmpc_rti_step_ipm(C.byref(d), *args, float(tol), int(max_iter), _stream(stream)),
                "rti_step_ipm")


def step_batched(descs, settings=None, stream=None):
    """gnmpc_step_batched over a list of StepDesc (see step_desc): every
    instance's linearize, condense and QP, run concurrently and joined back
    onto `stream`."""
    arr = (StepDesc * len(descs))(*descs)
    st = settings or default_admm_settings()
    s = lib().gnmpc_step_batched(arr, len(descs), C.byref(st), _stream(stream))
    if s != OK:
        raise GnmpcError(s, "step_batched: " + status_string(s))


def qp_info(t):
    """Decode a device info buffer (uint8 tensor of QP_INFO_BYTES) after a sync."""
    b = bytes(t.cpu().numpy().tobytes())
    return QpInfo.from_buffer_copy(b)


def lin_info(t):
    """Decode a linearization report (uint8 tensor of LIN_INFO_BYTES) after a sync."""
    return LinInfo.from_buffer_copy(bytes(t.cpu().numpy().tobytes()))
