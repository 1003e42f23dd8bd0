"""Torch-facing wrapper of the C ABI: contexts, compiled circuits and batches.

PyTorch supplies device memory (tensors) and the stream; the wrapper only marshals pointers
and sizes into the library, which runs every step in its own HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


def _ptr(t):
    return None if t is None else t.data_ptr()


def _f32(t, dev):
    if t is None:
        return None
    t = torch.as_tensor(t)
    return t.to(device=dev, dtype=torch.float32).contiguous()


def _aligned_bytes(nbytes, dev):
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=dev)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off, int(nbytes)


class Context:
    """One library context bound to a device and a HIP stream (default: torch's current one)."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        L.check(L.qp_ctx_create(device, self.stream.cuda_stream, C.byref(h)))
        self.h = h
        self.dev = torch.device("cuda", device)

    def use_stream(self, stream: torch.cuda.Stream):
        self.stream = stream
        L.check(L.qp_ctx_set_stream(self.h, stream.cuda_stream), self.h)

    def sync(self):
        L.check(L.qp_sync(self.h), self.h)

    def kernel_timing(self, on: bool = True):
        L.check(L.qp_ctx_enable_kernel_timing(self.h, 1 if on else 0), self.h)

    def last_kernel_ms(self) -> float:
        ms = C.c_float(0.0)
        L.check(L.qp_ctx_last_kernel_ms(self.h, C.byref(ms)), self.h)
        return float(ms.value)

    @property
    def cu_count(self):
        return L.qp_device_cu_count(self.h)

    def close(self):
        if self.h:
            L.qp_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_desc(circ):
    """qp_circuit_desc from any object with n, gates [(kind,q0,q1,param)], n_params, enc, out_qubits.
    Returns (desc, keepalive)."""
    n = int(circ.n)
    gates = (L.qp_gate * max(1, len(circ.gates)))()
    for i, (k, q0, q1, p) in enumerate(circ.gates):
        gates[i] = L.qp_gate(int(k), int(q0), int(q1), int(p))
    outs = (C.c_int32 * len(circ.out_qubits))(*[int(q) for q in circ.out_qubits])
    enc = circ.enc
    keep = [gates, outs]
    e = L.qp_encoding()
    e.kind, e.gate, e.scale = int(enc.kind), int(enc.gate), int(enc.scale)
    coords = getattr(enc, "coord_of_qubit", None)
    if coords is not None:
        ca = (C.c_int32 * n)(*[int(c) for c in coords])
        keep.append(ca)
        e.coord_of_qubit = ca
    if getattr(enc, "rff_B", None) is not None:
        B = np.ascontiguousarray(enc.rff_B, dtype=np.float32)
        W = np.ascontiguousarray(enc.rff_W, dtype=np.float32)
        keep += [B, W]
        e.n_features = B.shape[0]
        e.rff_B = B.ctypes.data_as(C.POINTER(C.c_float))
        e.rff_W = W.ctypes.data_as(C.POINTER(C.c_float))
    d = L.qp_circuit_desc()
    d.n_qubits, d.n_params, d.n_gates = n, int(circ.n_params), len(circ.gates)
    d.gates = gates
    d.enc = e
    d.n_out = len(circ.out_qubits)
    d.out_qubits = outs
    return d, keep


def maxwell_desc(loss):
    kind = int(getattr(loss, "kind", 0))
    return L.qp_maxwell_desc(kind, float(getattr(loss, "eps_r", 4.0)), float(getattr(loss, "x_interface", 0.0)))


class Circuit:
    """A compiled circuit (plan uploaded once)."""

    def __init__(self, ctx: Context, circ):
        self.ctx = ctx
        self.src = circ
        d, keep = make_desc(circ)
        h = C.c_void_p()
        L.check(L.qp_circuit_compile(ctx.h, C.byref(d), C.byref(h)), ctx.h)
        self.h = h
        self.n = int(circ.n)
        self.K = int(circ.n_params)
        self.m = len(circ.out_qubits)
        self._ws = {}

    def info(self, what: int) -> int:
        return int(L.qp_circuit_info(self.h, what))

    def set_launch(self, exchange_planes: int, wg_per_cu: int) -> None:
        L.check(L.qp_circuit_set_launch(self.h, int(exchange_planes), int(wg_per_cu)), self.ctx.h)

    def set_dense_chunk(self, points: int) -> None:
        L.check(L.qp_circuit_set_dense_chunk(self.h, int(points)), self.ctx.h)

    def workspace(self, P: int, flags: int = 0):
        nb = int(L.qp_workspace_bytes(self.h, int(P), int(flags) & (L.QP_FLAG_DENSE_MFMA | L.QP_FLAG_TUNE)))
        key = ("ws", nb)
        if key not in self._ws:
            self._ws = {key: _aligned_bytes(nb, self.ctx.dev)}
        return self._ws[key]

    def _inputs(self, params, points, angles, jac):
        dev = self.ctx.dev
        return _f32(params, dev), _f32(points, dev), _f32(angles, dev), _f32(jac, dev)

    def simulate(self, params, points=None, angles=None, jac=None, tangents=True, out=None, tan=None, flags=0):
        prm, pts, ang, jc = self._inputs(params, points, angles, jac)
        P = int((pts if pts is not None else ang).shape[0])
        dev = self.ctx.dev
        out = out if out is not None else torch.empty((P, self.m), dtype=torch.float32, device=dev)
        if tangents and tan is None:
            tan = torch.empty((P, self.m, 3), dtype=torch.float32, device=dev)
        _, wp, nb = self.workspace(P, flags)
        flags = flags | (0 if tangents else L.QP_FLAG_NO_TANGENTS)
        L.check(L.qp_simulate(self.ctx.h, self.h, _ptr(prm), _ptr(pts), _ptr(ang), _ptr(jc), P, _ptr(out),
                              _ptr(tan) if tangents else None, wp, nb, flags), self.ctx.h)
        return out, (tan if tangents else None)

    def vjp(self, params, points=None, d_out=None, d_tan=None, angles=None, jac=None, d_params=None, flags=0,
            input_grads=False):
        """d_params [K]; with input_grads=True (angle-given encoding) returns (d_params, d_angles [P,n],
        d_jac [P,n,3])."""
        prm, pts, ang, jc = self._inputs(params, points, angles, jac)
        P = int((pts if pts is not None else ang).shape[0])
        dev = self.ctx.dev
        d_out = _f32(d_out, dev)
        d_tan = _f32(d_tan, dev)
        d_params = d_params if d_params is not None else torch.empty(self.K, dtype=torch.float32, device=dev)
        d_ang = torch.empty((P, self.n), dtype=torch.float32, device=dev) if input_grads else None
        d_jac = torch.empty((P, self.n, 3), dtype=torch.float32, device=dev) if input_grads else None
        _, wp, nb = self.workspace(P, flags)
        L.check(L.qp_vjp(self.ctx.h, self.h, _ptr(prm), _ptr(pts), _ptr(ang), _ptr(jc), P, _ptr(d_out), _ptr(d_tan),
                         _ptr(d_params), _ptr(d_ang), _ptr(d_jac), wp, nb, flags), self.ctx.h)
        return (d_params, d_ang, d_jac) if input_grads else d_params

    def maxwell(self, params, points, loss, angles=None, jac=None, outputs=True, flags=0, bufs=None,
                input_grads=False):
        """Fused forward + tangents + Maxwell loss + adjoint gradient.  Returns
        dict(out, tan, loss (float64 [1]), grad (float32 [K])), plus d_angles [P,n] and d_jac [P,n,3]
        with input_grads=True (angle-given encoding)."""
        prm, pts, ang, jc = self._inputs(params, points, angles, jac)
        P = int((pts if pts is not None else ang).shape[0])
        dev = self.ctx.dev
        if bufs is None:
            bufs = {
                "out": torch.empty((P, self.m), dtype=torch.float32, device=dev) if outputs else None,
                "tan": torch.empty((P, self.m, 3), dtype=torch.float32, device=dev) if outputs else None,
                "loss": torch.empty(1, dtype=torch.float64, device=dev),
                "grad": torch.empty(self.K, dtype=torch.float32, device=dev),
            }
        if input_grads:
            bufs["d_angles"] = torch.empty((P, self.n), dtype=torch.float32, device=dev)
            bufs["d_jac"] = torch.empty((P, self.n, 3), dtype=torch.float32, device=dev)
        _, wp, nb = self.workspace(P, flags)
        md = maxwell_desc(loss)
        L.check(L.qp_maxwell_fused(self.ctx.h, self.h, _ptr(prm), _ptr(pts), _ptr(ang), _ptr(jc), P, C.byref(md),
                                   _ptr(bufs["out"]), _ptr(bufs["tan"]), _ptr(bufs["loss"]), _ptr(bufs["grad"]),
                                   _ptr(bufs.get("d_angles")), _ptr(bufs.get("d_jac")), wp, nb, flags), self.ctx.h)
        return bufs

    def maxwell_noalloc(self, params, points, loss, angles=None, jac=None, flags=0, bufs=None):
        """qp_maxwell_fused_noalloc: the same evaluation with the library's fixed scratch array
        instead of a workspace (the caller still provides inputs and outputs)."""
        prm, pts, ang, jc = self._inputs(params, points, angles, jac)
        P = int((pts if pts is not None else ang).shape[0])
        dev = self.ctx.dev
        if bufs is None:
            bufs = {"out": torch.empty((P, self.m), dtype=torch.float32, device=dev),
                    "tan": torch.empty((P, self.m, 3), dtype=torch.float32, device=dev),
                    "loss": torch.empty(1, dtype=torch.float64, device=dev),
                    "grad": torch.empty(self.K, dtype=torch.float32, device=dev)}
        md = maxwell_desc(loss)
        L.check(L.qp_maxwell_fused_noalloc(self.ctx.h, self.h, _ptr(prm), _ptr(pts), _ptr(ang), _ptr(jc), P,
                                           C.byref(md), _ptr(bufs["out"]), _ptr(bufs["tan"]), _ptr(bufs["loss"]),
                                           _ptr(bufs["grad"]), None, None, flags), self.ctx.h)
        return bufs

    def total_loss(self, params, points, ic_xy, desc, outputs=False, flags=0):
        """The paper's total loss (qp_total_loss): returns dict(terms (float64 [5]: total, phys, ic,
        sym, energy), grad (float32 [K]), and out/tan of the collocation points if outputs)."""
        dev = self.ctx.dev
        prm, pts = _f32(params, dev), _f32(points, dev)
        xy = _f32(ic_xy, dev)
        P, P0 = int(pts.shape[0]), int(xy.shape[0])
        r = {"terms": torch.empty(5, dtype=torch.float64, device=dev),
             "grad": torch.empty(self.K, dtype=torch.float32, device=dev),
             "out": torch.empty((P, self.m), dtype=torch.float32, device=dev) if outputs else None,
             "tan": torch.empty((P, self.m, 3), dtype=torch.float32, device=dev) if outputs else None}
        phys = desc.phys
        d = L.qp_total_loss_desc(maxwell_desc(phys), float(desc.w_ic), float(desc.w_sym), float(desc.w_energy),
                                 float(desc.ic_a))
        nb = int(L.qp_total_workspace_bytes(self.h, P, P0, int(phys.kind)))
        key = ("total", nb)
        if key not in self._ws:
            self._ws[key] = _aligned_bytes(nb, dev)
        _, wp, _ = self._ws[key]
        L.check(L.qp_total_loss(self.ctx.h, self.h, _ptr(prm), _ptr(pts), P, _ptr(xy), P0, C.byref(d),
                                _ptr(r["out"]), _ptr(r["tan"]), _ptr(r["terms"]), _ptr(r["grad"]), wp, nb, flags),
                self.ctx.h)
        return r

    def bloch(self, params, points=None, angles=None, precision=32):
        """Per-qubit Bloch vectors [P, n, 3] and Meyer-Wallach entanglement [P] of the output states."""
        dt = torch.float64 if precision == 64 else torch.float32
        dev = self.ctx.dev
        prm = torch.as_tensor(params).to(dev, dt).contiguous()
        pts = None if points is None else torch.as_tensor(points).to(dev, dt).contiguous()
        ang = None if angles is None else torch.as_tensor(angles).to(dev, dt).contiguous()
        P = int((pts if pts is not None else ang).shape[0])
        r = torch.empty((P, self.n, 3), dtype=dt, device=dev)
        mw = torch.empty(P, dtype=dt, device=dev)
        _, wp, nb = self.plain_workspace(P, precision)
        L.check(L.qp_bloch(self.ctx.h, self.h, precision, _ptr(prm), _ptr(pts), _ptr(ang), P, _ptr(r), _ptr(mw), wp,
                           nb), self.ctx.h)
        return r, mw

    def energy_profile(self, params, t, xg, yg, loss=None, flags=0):
        """U(t_i) = sum over the grid xg x yg of (eps E^2 + Hx^2 + Hy^2) / 2, float64 [Nt]."""
        dev = self.ctx.dev
        prm, tt, xx, yy = _f32(params, dev), _f32(t, dev), _f32(xg, dev), _f32(yg, dev)
        Nt, Nx, Ny = int(tt.shape[0]), int(xx.shape[0]), int(yy.shape[0])
        U = torch.empty(Nt, dtype=torch.float64, device=dev)
        nb = int(L.qp_energy_workspace_bytes(self.h, Nt, Nx, Ny))
        key = ("energy", nb)
        if key not in self._ws:
            self._ws[key] = _aligned_bytes(nb, dev)
        _, wp, _ = self._ws[key]
        md = maxwell_desc(loss) if loss is not None else None
        L.check(L.qp_energy_profile(self.ctx.h, self.h, _ptr(prm), _ptr(tt), Nt, _ptr(xx), Nx, _ptr(yy), Ny,
                                    C.byref(md) if md is not None else None, _ptr(U), wp, nb, flags), self.ctx.h)
        return U

    # ---- plain baseline -------------------------------------------------------------------
    def plain_workspace(self, P, precision):
        nb = int(L.qp_plain_workspace_bytes(self.h, int(P), int(precision)))
        key = ("plain", nb)
        if key not in self._ws:
            self._ws[key] = _aligned_bytes(nb, self.ctx.dev)
        return self._ws[key]

    def plain_eval(self, params, points, precision=32, h=None, tangents=True):
        dt = torch.float64 if precision == 64 else torch.float32
        dev = self.ctx.dev
        prm = torch.as_tensor(params).to(dev, dt).contiguous()
        pts = torch.as_tensor(points).to(dev, dt).contiguous()
        P = int(pts.shape[0])
        h = h if h is not None else (1e-5 if precision == 64 else 2.0 ** -7)
        out = torch.empty((P, self.m), dtype=dt, device=dev)
        tan = torch.empty((P, self.m, 3), dtype=dt, device=dev) if tangents else None
        _, wp, nb = self.plain_workspace(P, precision)
        L.check(L.qp_plain_eval(self.ctx.h, self.h, precision, _ptr(prm), _ptr(pts), P, float(h), _ptr(out),
                                _ptr(tan), wp, nb), self.ctx.h)
        return out, tan

    def plain_maxwell_fd(self, params, points, loss, precision=32, h=None, h_param=None, k_begin=0, k_end=None):
        dt = torch.float64 if precision == 64 else torch.float32
        dev = self.ctx.dev
        prm = torch.as_tensor(params).to(dev, dt).contiguous()
        pts = torch.as_tensor(points).to(dev, dt).contiguous()
        P = int(pts.shape[0])
        h = h if h is not None else (1e-5 if precision == 64 else 2.0 ** -7)
        h_param = h_param if h_param is not None else (1e-5 if precision == 64 else 2.0 ** -7)
        k_end = self.K if k_end is None else k_end
        lo = torch.empty(1, dtype=torch.float64, device=dev)
        dp = torch.zeros(self.K, dtype=dt, device=dev)
        _, wp, nb = self.plain_workspace(P, precision)
        md = maxwell_desc(loss)
        L.check(L.qp_plain_maxwell_fd(self.ctx.h, self.h, precision, _ptr(prm), _ptr(pts), P, C.byref(md), float(h),
                                      float(h_param), int(k_begin), int(k_end), _ptr(lo), _ptr(dp), wp, nb),
                self.ctx.h)
        return lo, dp

    def close(self):
        if self.h:
            L.qp_circuit_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many circuits with their own point sets, evaluated by one persistent launch."""

    def __init__(self, ctx: Context, circuits, P):
        self.ctx = ctx
        descs = (L.qp_circuit_desc * len(circuits))()
        self._keep = []
        for i, c in enumerate(circuits):
            d, keep = make_desc(c)
            descs[i] = d
            self._keep.append(keep)
        Ps = (C.c_int64 * len(P))(*[int(p) for p in P])
        h = C.c_void_p()
        L.check(L.qp_batch_compile(ctx.h, len(circuits), descs, Ps, C.byref(h)), ctx.h)
        self.h = h
        self.circuits = circuits
        self.P = [int(p) for p in P]
        nb = int(L.qp_batch_workspace_bytes(h))
        self._ws = _aligned_bytes(nb, ctx.dev)

    def info(self, what):
        return int(L.qp_batch_info(self.h, what))

    def io(self, params_list, points_list, outputs=True):
        dev = self.ctx.dev
        bufs = []
        arr = (L.qp_batch_io * len(self.circuits))()
        for i, c in enumerate(self.circuits):
            m = len(c.out_qubits)
            P = self.P[i]
            b = {"params": _f32(params_list[i], dev), "points": _f32(points_list[i], dev),
                 "out": torch.empty((P, m), dtype=torch.float32, device=dev) if outputs else None,
                 "tan": torch.empty((P, m, 3), dtype=torch.float32, device=dev) if outputs else None,
                 "loss": torch.empty(1, dtype=torch.float64, device=dev),
                 "grad": torch.empty(int(c.n_params), dtype=torch.float32, device=dev)}
            arr[i] = L.qp_batch_io(_ptr(b["params"]), _ptr(b["points"]), _ptr(b["out"]), _ptr(b["tan"]),
                                   _ptr(b["loss"]), _ptr(b["grad"]))
            bufs.append(b)
        return arr, bufs

    def run(self, arr, loss, flags=0, graph=False):
        md = maxwell_desc(loss)
        _, wp, nb = self._ws
        fn = L.qp_batch_graph_launch if graph else L.qp_batch_run
        L.check(fn(self.ctx.h, self.h, arr, C.byref(md), wp, nb, flags), self.ctx.h)

    def close(self):
        if self.h:
            L.qp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
